// Per-frequency shifted Hessenberg solves: one wavefront per tile of
// frequencies of one request.
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
// its step: y_k = b_k / r, b_{0..k-1} -= R(0..k-1, k) y_k.  R is never
// stored.  Then X = Z y is formed by applying the rotations in increasing
// order, which is the first-order linear recurrence
//
//     t_0 = y_0,  t_k = -c_k t_{k-1} + conj(s_k) y_k,
//     x_{k-1} = s_k t_{k-1} + c_k y_k,  x_{n-1} = t_{n-1} ,
//
// evaluated as a Kogge-Stone scan across lanes.  Finally G = Ct^T X + D with a
// reduce-scatter over the 64 lanes.
//
// Lane layout: row i lives on lane i % 64 in register slice i / 64 (R slices,
// n <= 64 R); each lane holds its rows' carry entry (column being rotated),
// right-hand-side rows (m <= MM complex) and, after the sweep, its rows' y
// and rotation parameters.  The sweep reads H one column per step, right to
// left, straight from the packed column-major layout (the next column is
// loaded while the current one is used); every frequency of a request reads
// the same H, which stays in L2.
#include <cfloat>
#include <cmath>

#include "lti_kernels.h"

namespace lti {

namespace {

constexpr int kWaves = 4;  // wavefronts per workgroup, one tile each

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
__device__ __forceinline__ double sqrt_t(double x) { return sqrt(x); }
__device__ __forceinline__ float sqrt_t(float x) { return sqrtf(x); }

template <typename T>
struct Limits;
template <>
struct Limits<double> {
  static constexpr double eps = DBL_EPSILON / 2;
};

// Register state of one frequency's solve.
template <typename T, int R, int MM>
struct Sweep {
  T cr[R], ci[R];            // carry column (real, imag)
  T br[R][MM], bi[R][MM];    // right-hand side, then y, then x
  T rc[R], rsr[R], rsi[R];   // rotation k stored on row k (row 0: unused)
  T dmin, dmax;              // extreme |R(k,k)|
  bool singular;
};

// Givens RQ sweep fused with back-substitution.  On entry br/bi hold the
// right-hand side rows; on exit they hold y.
template <typename T, int R, int MM>
__device__ __forceinline__ void givens_sweep(const T* __restrict__ H, int n, T w, Sweep<T, R, MM>& st) {
  const int lane = threadIdx.x & 63;
  st.dmin = (T)INFINITY;
  st.dmax = (T)0;
  st.singular = false;
  {
    const T* col = H + hoff(n - 1);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      const T h = (i < n) ? col[i] : (T)0;
      st.cr[r] = -h;
      st.ci[r] = (i == n - 1) ? w : (T)0;
      st.rc[r] = (T)0;
      st.rsr[r] = (T)1;
      st.rsi[r] = (T)0;
    }
  }
  T hc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) hc[r] = (T)0;
  if (n >= 2) {
    const T* col = H + hoff(n - 2);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      if (i <= n - 1) hc[r] = col[i];
    }
  }

#pragma unroll
  for (int s = R - 1; s >= 0; --s) {
    if (64 * s > n - 1) continue;  // no pivot row in this slice
    const int khi = (n - 1 < 64 * s + 63) ? n - 1 : 64 * s + 63;
    const int klo = (64 * s > 1) ? 64 * s : 1;
    for (int k = khi; k >= klo; --k) {
      const int kl = k - 64 * s;
      // prefetch column k-2, rows 0..k-1, for the next step
      T hn[R];
#pragma unroll
      for (int t = 0; t < R; ++t) hn[t] = (T)0;
      if (k >= 2) {
        const T* coln = H + hoff(k - 2);
#pragma unroll
        for (int t = 0; t <= s; ++t) {
          const int i = lane + 64 * t;
          if (i <= k - 1) hn[t] = coln[i];
        }
      }
      const T ar = readlane(st.cr[s], kl);
      const T ai = readlane(st.ci[s], kl);
      const T beta = -readlane(hc[s], kl);
      const T nrm2 = ar * ar + ai * ai + beta * beta;
      T rinv, c, sr, si, rkk;
      if (nrm2 > (T)0) {
        rinv = rsqrt_t(nrm2);
        c = beta * rinv;
        sr = ar * rinv;
        si = ai * rinv;
        rkk = nrm2 * rinv;
      } else {  // column already zero: identity rotation, R(k,k) = 0
        rinv = (T)INFINITY;
        c = (T)0;
        sr = (T)1;
        si = (T)0;
        rkk = (T)0;
        st.singular = true;
      }
      st.dmin = fmin(st.dmin, rkk);
      st.dmax = fmax(st.dmax, rkk);
      T yr[MM], yi[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        yr[j] = readlane(st.br[s][j], kl) * rinv;
        yi[j] = readlane(st.bi[s][j], kl) * rinv;
      }
#pragma unroll
      for (int t = 0; t <= s; ++t) {
        if (t < s || lane < kl) {
          const int i = lane + 64 * t;
          const T cr_ = st.cr[t], ci_ = st.ci[t];
          const T orr = -hc[t];
          const T oi = (i == k - 1) ? w : (T)0;
          // new column k (final R(i, k)) and new carry (column k-1)
          const T nkr = c * orr + sr * cr_ + si * ci_;
          const T nki = c * oi + sr * ci_ - si * cr_;
          st.cr[t] = sr * orr - si * oi - c * cr_;
          st.ci[t] = sr * oi + si * orr - c * ci_;
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            st.br[t][j] -= nkr * yr[j] - nki * yi[j];
            st.bi[t][j] -= nkr * yi[j] + nki * yr[j];
          }
        }
      }
      if (lane == kl) {
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          st.br[s][j] = yr[j];
          st.bi[s][j] = yi[j];
        }
        st.rc[s] = c;
        st.rsr[s] = sr;
        st.rsi[s] = si;
      }
#pragma unroll
      for (int t = 0; t < R; ++t) hc[t] = hn[t];
    }
  }
  // row 0: R(0,0) is the carry entry itself (complex)
  {
    const T ar = readlane(st.cr[0], 0);
    const T ai = readlane(st.ci[0], 0);
    const T d = ar * ar + ai * ai;
    const T dinv = (T)1 / d;  // inf when singular
    if (!(d > (T)0)) st.singular = true;
    const T r0 = sqrt_t(d);
    st.dmin = fmin(st.dmin, r0);
    st.dmax = fmax(st.dmax, r0);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const T xr = st.br[0][j], xi = st.bi[0][j];
        st.br[0][j] = (xr * ar + xi * ai) * dinv;
        st.bi[0][j] = (xi * ar - xr * ai) * dinv;
      }
    }
  }
}

// x := Z y, in place in br/bi (see the recurrence at the top of the file).
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
    // element i: t -> a t + u
    T a;
    T ur[MM], ui[MM];
    if (i == 0 || i >= n) {
      a = (T)0;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        ur[j] = (i == 0) ? st.br[s][j] : (T)0;
        ui[j] = (i == 0) ? st.bi[s][j] : (T)0;
      }
    } else {
      a = -st.rc[s];
      const T sr = st.rsr[s], si = st.rsi[s];
#pragma unroll
      for (int j = 0; j < MM; ++j) {  // conj(s) * y
        ur[j] = sr * st.br[s][j] + si * st.bi[s][j];
        ui[j] = sr * st.bi[s][j] - si * st.br[s][j];
      }
    }
    // inclusive scan: (a, u) o (a', u') = (a a', a u' + u)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const T ap = __shfl_up(a, d, 64);
      T upr[MM], upi[MM];
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        upr[j] = __shfl_up(ur[j], d, 64);
        upi[j] = __shfl_up(ui[j], d, 64);
      }
      if (lane >= d) {
#pragma unroll
        for (int j = 0; j < MM; ++j) {
          ur[j] = a * upr[j] + ur[j];
          ui[j] = a * upi[j] + ui[j];
        }
        a = a * ap;
      }
    }
    T tr[MM], ti[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      tr[j] = a * tinr[j] + ur[j];
      ti[j] = a * tini[j] + ui[j];
    }
    // rotation and y of row i+1
    T nc = __shfl_down(st.rc[s], 1, 64);
    T nsr = __shfl_down(st.rsr[s], 1, 64);
    T nsi = __shfl_down(st.rsi[s], 1, 64);
    T nyr[MM], nyi[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      nyr[j] = __shfl_down(st.br[s][j], 1, 64);
      nyi[j] = __shfl_down(st.bi[s][j], 1, 64);
    }
    if (s + 1 < R) {
      // lane 63 takes row 64(s+1) from the next slice
      const T c0 = readlane(st.rc[s + 1 < R ? s + 1 : s], 0);
      const T s0r = readlane(st.rsr[s + 1 < R ? s + 1 : s], 0);
      const T s0i = readlane(st.rsi[s + 1 < R ? s + 1 : s], 0);
      if (lane == 63) {
        nc = c0;
        nsr = s0r;
        nsi = s0i;
      }
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const T y0r = readlane(st.br[s + 1 < R ? s + 1 : s][j], 0);
        const T y0i = readlane(st.bi[s + 1 < R ? s + 1 : s][j], 0);
        if (lane == 63) {
          nyr[j] = y0r;
          nyi[j] = y0i;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      tinr[j] = readlane(tr[j], 63);
      tini[j] = readlane(ti[j], 63);
    }
    if (i < n - 1) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {  // x_i = s_{i+1} t_i + c_{i+1} y_{i+1}
        st.br[s][j] = nsr * tr[j] - nsi * ti[j] + nc * nyr[j];
        st.bi[s][j] = nsr * ti[j] + nsi * tr[j] + nc * nyi[j];
      }
    } else if (i == n - 1) {
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        st.br[s][j] = tr[j];
        st.bi[s][j] = ti[j];
      }
    }
  }
}

// One halving stage of the reduce-scatter: lanes whose bit D is set keep the
// upper H entries and send the lower ones to their partner (and vice versa).
template <int H, int D>
__device__ __forceinline__ void rs_stage(double (&vr)[16], double (&vi)[16]) {
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

// Sum of v over the 64 lanes for 16 complex values at once: after the call
// lane l holds the total of index l >> 2 in vr[0], vi[0].
__device__ __forceinline__ void reduce_scatter16(double (&vr)[16], double (&vi)[16]) {
  rs_stage<8, 32>(vr, vi);
  rs_stage<4, 16>(vr, vi);
  rs_stage<2, 8>(vr, vi);
  rs_stage<1, 4>(vr, vi);
  vr[0] += __shfl_xor(vr[0], 2, 64);
  vi[0] += __shfl_xor(vi[0], 2, 64);
  vr[0] += __shfl_xor(vr[0], 1, 64);
  vi[0] += __shfl_xor(vi[0], 1, 64);
}

// G = Ct^T X + D for one frequency, X in xr/xi (rows lane + 64 r).
template <int R, int MM>
__device__ __forceinline__ void write_output(const ReqDesc& rd, const double (&xr)[R][MM],
                                             const double (&xi)[R][MM], double* __restrict__ G) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m, p = rd.p;
  constexpr int PC = 16 / MM;  // rows of G per pass
  for (int a0 = 0; a0 < p; a0 += PC) {
    double vr[16], vi[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) vr[q] = vi[q] = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
      if (i < n) {
#pragma unroll
        for (int q = 0; q < PC; ++q) {
          const int a = a0 + q;
          const double cq = (a < p) ? rd.Ct[(size_t)i * p + a] : 0.0;
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            vr[q * MM + j] += cq * xr[r][j];
            vi[q * MM + j] += cq * xi[r][j];
          }
        }
      }
    }
    reduce_scatter16(vr, vi);
    if ((lane & 3) == 0) {
      const int idx = lane >> 2;
      const int a = a0 + idx / MM;
      const int j = idx % MM;
      if (a < p && j < m) {
        double2 g;
        g.x = vr[0] + rd.D[(size_t)a * m + j];
        g.y = vi[0];
        reinterpret_cast<double2*>(G)[(size_t)a * m + j] = g;
      }
    }
  }
}

__device__ __forceinline__ int xcd_swizzle(int b, int nb) {
  // Workgroups are dealt to the 8 XCDs round-robin; renumber them so that each
  // XCD works on a contiguous range of tiles (tiles of one request share H in
  // that XCD's L2).
  const int per = nb / 8, rem = nb % 8;
  const int xcd = b % 8, pos = b / 8;
  return (xcd < rem) ? xcd * (per + 1) + pos : rem * (per + 1) + (xcd - rem) * per + pos;
}

template <int R, int MM>
__device__ void solve_fp64(const ReqDesc& rd, int64_t k) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m;
  const double w = rd.omega[k];
  Sweep<double, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < m) ? rd.Bt[(size_t)i * m + j] : 0.0;
      st.bi[r][j] = 0.0;
    }
  }
  givens_sweep<double, R, MM>(rd.H, n, w, st);
  apply_rotations<double, R, MM>(n, st);
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output<R, MM>(rd, st.br, st.bi, G);
  if (rd.info && lane == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)(Limits<double>::eps * (st.dmax / st.dmin));
    inf.iters = 1;
    inf.path = st.singular ? LTI_PATH_SINGULAR : LTI_PATH_FP64;
    inf.reserved = 0;
    rd.info[k] = inf;
  }
}

// ---------------------------------------------------------------- refined

// Wave-wide sum and max.
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

// r = Bt - (j w X - H X), float64, rows lane + 64 t.
template <int R, int MM>
__device__ __forceinline__ void residual64(const ReqDesc& rd, double w, const double (&xr)[R][MM],
                                           const double (&xi)[R][MM], double (&rr)[R][MM],
                                           double (&ri)[R][MM]) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m;
#pragma unroll
  for (int t = 0; t < R; ++t) {
    const int i = lane + 64 * t;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double b = (i < n && j < m) ? rd.Bt[(size_t)i * m + j] : 0.0;
      rr[t][j] = b + w * xi[t][j];
      ri[t][j] = -w * xr[t][j];
    }
  }
#pragma unroll
  for (int sj = 0; sj < R; ++sj) {
    if (64 * sj >= n) break;
    const int jend = (n - 64 * sj < 64) ? n - 64 * sj : 64;
    for (int jl = 0; jl < jend; ++jl) {
      const int jc = 64 * sj + jl;  // column of H
      const double* col = rd.H + hoff(jc);
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
          const double h = col[i];
#pragma unroll
          for (int j = 0; j < MM; ++j) {
            rr[t][j] += h * xjr[j];
            ri[t][j] += h * xji[j];
          }
        }
      }
    }
  }
}

template <int R, int MM>
__device__ void solve_refined(const ReqDesc& rd, int64_t k) {
  const int lane = threadIdx.x & 63;
  const int n = rd.n, m = rd.m;
  const double w = rd.omega[k];
  const float wf = (float)w;
  const double tol = 0.1 * ((rd.rtol > 0.0) ? rd.rtol : 1e-10);
  constexpr int kMaxIters = 6;

  double xr[R][MM], xi[R][MM];
  Sweep<float, R, MM> st;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      st.br[r][j] = (i < n && j < m) ? rd.Bt32[(size_t)i * m + j] : 0.0f;
      st.bi[r][j] = 0.0f;
    }
  }
  givens_sweep<float, R, MM>(rd.H32, n, wf, st);
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
  int path = LTI_PATH_REFINED;
  double est = 1.0;
  bool ok = false;
  if (st.singular || !(dprev < INFINITY)) {
    path = LTI_PATH_FALLBACK;
  } else {
    for (int it = 0; it < kMaxIters; ++it) {
      double rr[R][MM], ri[R][MM];
      residual64<R, MM>(rd, w, xr, xi, rr, ri);
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
      givens_sweep<float, R, MM>(rd.H32, n, wf, st);
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
      if (!(dn < INFINITY) || !(xn > 0.0)) break;  // non-finite: fall back
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
    if (!ok) path = LTI_PATH_FALLBACK;
  }
  bool singular = false;
  if (path == LTI_PATH_FALLBACK) {
    Sweep<double, R, MM> sd;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int i = lane + 64 * r;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        sd.br[r][j] = (i < n && j < m) ? rd.Bt[(size_t)i * m + j] : 0.0;
        sd.bi[r][j] = 0.0;
      }
    }
    givens_sweep<double, R, MM>(rd.H, n, w, sd);
    apply_rotations<double, R, MM>(n, sd);
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        xr[r][j] = sd.br[r][j];
        xi[r][j] = sd.bi[r][j];
      }
    singular = sd.singular;
    est = Limits<double>::eps * (sd.dmax / sd.dmin);
    if (singular) path = LTI_PATH_SINGULAR;
  }
  double* G = rd.G + (size_t)k * rd.p * m * 2;
  write_output<R, MM>(rd, xr, xi, G);
  if (rd.info && lane == 0) {
    lti_point_info inf;
    inf.est_rel_err = (float)est;
    inf.iters = (uint8_t)iters;
    inf.path = (uint8_t)path;
    inf.reserved = 0;
    rd.info[k] = inf;
  }
}

template <int PREC, int R, int MM>
__global__ __launch_bounds__(64 * kWaves) void sweep_kernel(const TileDesc* __restrict__ tiles, int ntiles) {
  // the tile index is uniform per wavefront; say so, so that the descriptor
  // loads become scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = xcd_swizzle(blockIdx.x, gridDim.x) * kWaves + wave;
  if (tile >= ntiles) return;
  const TileDesc td = tiles[tile];
  const ReqDesc rd = *td.rd;
  for (uint32_t f = 0; f < td.count; ++f) {
    const int64_t k = (int64_t)td.start + f;
    if (PREC == LTI_PREC_FP64)
      solve_fp64<R, MM>(rd, k);
    else
      solve_refined<R, MM>(rd, k);
  }
}

using KernelFn = void (*)(const TileDesc*, int);

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

hipError_t launch_sweep(int kclass, const TileDesc* tiles, int ntiles, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  if (kclass < 0 || kclass >= kNumSweepClasses) return hipErrorInvalidValue;
  const int mi = kclass % kNumRhsClasses;
  const int ri = (kclass / kNumRhsClasses) % kNumRowClasses;
  const int prec = kclass / (kNumRhsClasses * kNumRowClasses);
  const KernelFn fn = prec == LTI_PREC_FP64 ? pick<LTI_PREC_FP64>(ri, mi) : pick<LTI_PREC_REFINED>(ri, mi);
  const int blocks = (ntiles + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(fn, dim3(blocks), dim3(64 * kWaves), 0, s, tiles, ntiles);
  return hipGetLastError();
}

}  // namespace lti
