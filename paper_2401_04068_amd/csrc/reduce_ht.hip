// Hessenberg-triangular reduction of a descriptor system (E, A, B, C):
// orthogonal Q, Z with Q^T A Z = H upper Hessenberg and Q^T E Z = T upper
// triangular (Golub & Van Loan, Matrix Computations, 4th ed., Alg. 7.7.1;
// the first stage of Moler and Stewart's QZ algorithm).  Then
//
//     G(s) = C (s E - A)^{-1} B + D = (C Z) (s T - H)^{-1} (Q^T B) + D ,
//
// and every point costs one shifted solve with the Hessenberg matrix s T - H.
//
// One workgroup per model; the augmented matrix W = [[A, B], [C, *]] and E
// live column-major in the job's global work area (L2-resident for the sizes
// served, n <= 256).
//
// 1. QR of E by Householder reflectors from the left, applied to E and to the
//    rows of W (A and B).
// 2. For each column j of A, rows n-1 .. j+2 are zeroed bottom-up by Givens
//    rotations of rows (i-1, i) (applied to W and E); each creates one
//    nonzero E(i, i-1), removed at once by a Givens rotation of columns
//    (i-1, i) (applied to E, and to W including the C rows).  The row
//    rotations of column j only depend on column j, which column rotations
//    never touch, so one thread computes all of them first.  A step's column
//    rotation depends on E(i-1, i-1), E(i-1, i), E(i, i), which the previous
//    step changed; the thread that applies the previous step's 2 x 2 blocks
//    (and E's row i-1 of its column rotation) has exactly those values and
//    publishes the next step's column rotation, so each step needs one
//    barrier.
#include <hip/hip_runtime.h>

#include <cmath>

#include "lti_kernels.h"

namespace lti {
namespace {

constexpr int kHTThreads = 256;

__device__ __forceinline__ int ld_w(int n, int p) { return (n + p) | 1; }
__device__ __forceinline__ int ld_e(int n) { return n | 1; }

// Givens pair (c, s) with [c s; -s c] [a; b] = [r; 0], r >= 0.
__device__ __forceinline__ void givens(double a, double b, double& c, double& s) {
  const double r = hypot(a, b);
  if (r == 0.0) {
    c = 1.0;
    s = 0.0;
  } else {
    c = a / r;
    s = b / r;
  }
}

// Column rotation of step i from E(i-1, i-1), E(i-1, i), E(i, i) (values
// before step i) and step i's row rotation (c, s): after the row rotation
// E(i, i-1) = -s E(i-1, i-1) and E(i, i) = -s E(i-1, i) + c E(i, i); the
// column rotation [col_{i-1} col_i] [cz sz; -sz cz] zeroes the first.
__device__ __forceinline__ void col_rot(double e00, double e01, double e11, double c, double s, double& cz,
                                        double& sz) {
  const double f = -s * e00;
  const double g = fma(-s, e01, c * e11);
  const double r = hypot(f, g);
  if (r == 0.0) {
    cz = 1.0;
    sz = 0.0;
  } else {
    cz = g / r;
    sz = f / r;
  }
}

struct HTShared {
  double rc[kMaxN], rs[kMaxN];  // row rotations of the current column, by i
  double x[kMaxN];              // the column being reduced (one thread)
  double cz[2], sz[2];          // the next step's column rotation (double-buffered)
  double red[kHTThreads / 64];
  double v[kMaxN];
  double tau;
};

__global__ __launch_bounds__(kHTThreads) void hess_tri_kernel(const ReduceLaunch L) {
  __shared__ HTShared S;
  const ReduceJob job = L.jobs[blockIdx.x];
  const ModelIn in(job);
  const ReducedModel& o = job.out;
  const int n = o.n, m = o.m, p = o.p;
  const int ldw = ld_w(n, p), lde = ld_e(n);
  const int nrow = n + p, ncol = n + m;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double* W = job.work;
  double* E = job.work + (size_t)ldw * ncol;
  auto w = [&](int i, int c) -> double& { return W[(size_t)i + (size_t)ldw * c]; };
  auto e = [&](int i, int c) -> double& { return E[(size_t)i + (size_t)lde * c]; };

  for (int idx = tid; idx < nrow * ncol; idx += kHTThreads) {
    const int i = idx % nrow, c = idx / nrow;
    double x = 0.0;
    if (i < n)
      x = c < n ? in.a(i, c) : in.b(i, c - n);
    else if (c < n)
      x = in.c(i - n, c);
    w(i, c) = x;
  }
  for (int idx = tid; idx < n * n; idx += kHTThreads) e(idx % n, idx / n) = in.e(idx % n, idx / n);
  __syncthreads();

  // 1. E = Q1 R: reflector k zeroes E(k+1 .., k); applied to E and W's rows
  for (int k = 0; k + 1 < n; ++k) {
    double ss = 0.0;
    for (int i = k + 1 + tid; i < n; i += kHTThreads) {
      const double x = e(i, k);
      ss = fma(x, x, ss);
    }
    for (int d = 32; d >= 1; d >>= 1) ss += __shfl_xor(ss, d, 64);
    if (lane == 0) S.red[wv] = ss;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int q = 0; q < kHTThreads / 64; ++q) t += S.red[q];
      const double alpha = e(k, k);
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (t != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, t));
        beta = alpha >= 0.0 ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      S.tau = tau;
      S.v[k] = 1.0;
      S.x[0] = scale;
      S.x[1] = beta;
    }
    __syncthreads();
    const double tau = S.tau, scale = S.x[0], beta = S.x[1];
    for (int i = k + 1 + tid; i < n; i += kHTThreads) S.v[i] = e(i, k) * scale;
    __syncthreads();
    if (tid == 0) e(k, k) = beta;
    for (int i = k + 1 + tid; i < n; i += kHTThreads) e(i, k) = 0.0;
    if (tau != 0.0) {
      // columns k+1 .. n-1 of E, then all n + m columns of W (rows k .. n-1)
      for (int c = tid; c < (n - k - 1) + ncol; c += kHTThreads) {
        double* col = c < n - k - 1 ? &e(0, k + 1 + c) : &w(0, c - (n - k - 1));
        double s = 0.0;
        for (int i = k; i < n; ++i) s = fma(S.v[i], col[i], s);
        s *= tau;
        for (int i = k; i < n; ++i) col[i] = fma(-S.v[i], s, col[i]);
      }
    }
    __syncthreads();
  }

  // 2. Givens chase, column by column
  for (int j = 0; j + 2 < n; ++j) {
    if (tid == 0) {
      // row rotations of column j, bottom-up
      for (int i = j + 1; i < n; ++i) S.x[i] = w(i, j);
      for (int i = n - 1; i >= j + 2; --i) {
        double c, s;
        givens(S.x[i - 1], S.x[i], c, s);
        S.rc[i] = c;
        S.rs[i] = s;
        S.x[i - 1] = fma(c, S.x[i - 1], s * S.x[i]);
        S.x[i] = 0.0;
      }
      // the first step's column rotation
      const int i = n - 1;
      double cz, sz;
      col_rot(e(i - 1, i - 1), e(i - 1, i), e(i, i), S.rc[i], S.rs[i], cz, sz);
      S.cz[i & 1] = cz;
      S.sz[i & 1] = sz;
    }
    __syncthreads();
    for (int i = n - 1; i >= j + 2; --i) {
      const double c = S.rc[i], s = S.rs[i];
      const double cz = S.cz[i & 1], sz = S.sz[i & 1];
      // (R) rows i-1, i: W columns j+1 .. ncol-1 and E columns i+1 .. n-1,
      //     both without columns i-1, i;
      // (C) columns i-1, i: W rows 0 .. nrow-1 and E rows 0 .. i-2, both
      //     without rows i-1, i (E's row i-2 belongs to the block thread);
      // (X) the two 2 x 2 blocks and E's row i-2, one thread, which then
      //     publishes the next step's column rotation.
      const int nRw = ncol - (j + 1) - 2;       // W columns of (R)
      const int nRe = n - 1 - i;                // E columns of (R)
      const int nCw = nrow - 2;                 // W rows of (C)
      const int nCe = i >= 3 ? i - 2 : 0;       // E rows 0 .. i-3 of (C)
      const int total = nRw + nRe + nCw + nCe;
      for (int t = tid; t < total; t += kHTThreads) {
        if (t < nRw) {
          int cc = j + 1 + t;
          if (cc >= i - 1) cc += 2;  // skip columns i-1, i
          const double a = w(i - 1, cc), b = w(i, cc);
          w(i - 1, cc) = fma(c, a, s * b);
          w(i, cc) = fma(-s, a, c * b);
        } else if (t < nRw + nRe) {
          const int cc = i + 1 + (t - nRw);
          const double a = e(i - 1, cc), b = e(i, cc);
          e(i - 1, cc) = fma(c, a, s * b);
          e(i, cc) = fma(-s, a, c * b);
        } else if (t < nRw + nRe + nCw) {
          int r = t - nRw - nRe;
          if (r >= i - 1) r += 2;  // skip rows i-1, i
          const double a = w(r, i - 1), b = w(r, i);
          w(r, i - 1) = fma(cz, a, -sz * b);
          w(r, i) = fma(sz, a, cz * b);
        } else {
          const int r = t - nRw - nRe - nCw;  // 0 .. i-3
          const double a = e(r, i - 1), b = e(r, i);
          e(r, i - 1) = fma(cz, a, -sz * b);
          e(r, i) = fma(sz, a, cz * b);
        }
      }
      if (tid == kHTThreads - 1) {
        // W block: row rotation, then column rotation
        {
          const double a00 = w(i - 1, i - 1), a01 = w(i - 1, i), a10 = w(i, i - 1), a11 = w(i, i);
          const double r00 = fma(c, a00, s * a10), r01 = fma(c, a01, s * a11);
          const double r10 = fma(-s, a00, c * a10), r11 = fma(-s, a01, c * a11);
          w(i - 1, i - 1) = fma(cz, r00, -sz * r01);
          w(i - 1, i) = fma(sz, r00, cz * r01);
          w(i, i - 1) = fma(cz, r10, -sz * r11);
          w(i, i) = fma(sz, r10, cz * r11);
        }
        // E block (E(i, i-1) = 0 before; exactly 0 after)
        const double e00 = e(i - 1, i - 1), e01 = e(i - 1, i), e11 = e(i, i);
        const double r00 = c * e00, r01 = fma(c, e01, s * e11);
        const double r11 = fma(-s, e01, c * e11);
        const double n00 = fma(cz, r00, -sz * r01);
        const double n01 = fma(sz, r00, cz * r01);
        const double n11 = fma(sz, -s * e00, cz * r11);
        e(i - 1, i - 1) = n00;
        e(i - 1, i) = n01;
        e(i, i - 1) = 0.0;
        e(i, i) = n11;
        // E's row i-2 of the column rotation, and the next step's rotation
        if (i - 2 >= 0) {
          const double a = e(i - 2, i - 1), b = e(i - 2, i);
          const double na = fma(cz, a, -sz * b);
          e(i - 2, i - 1) = na;
          e(i - 2, i) = fma(sz, a, cz * b);
          if (i - 1 >= j + 2) {
            double cz2, sz2;
            col_rot(e(i - 2, i - 2), na, n00, S.rc[i - 1], S.rs[i - 1], cz2, sz2);
            S.cz[(i - 1) & 1] = cz2;
            S.sz[(i - 1) & 1] = sz2;
          }
        }
      }
      __syncthreads();
    }
    // column j of A: its reduced values (computed by the row rotations above)
    for (int i = j + 1 + tid; i < n; i += kHTThreads) w(i, j) = S.x[i];
    __syncthreads();
  }

  // H (packed Hessenberg), T (packed upper triangular), Q^T B, (C Z)^T, D
  for (int jj = 0; jj < n; ++jj) {
    const int len = jj + 2 < n ? jj + 2 : n;
    const int64_t off = hoff(jj);
    for (int i = tid; i < len; i += kHTThreads) {
      const double x = w(i, jj);
      o.H[off + i] = x;
      o.H32[off + i] = (float)x;
    }
    const int64_t toff = (int64_t)jj * (jj + 1) / 2;
    for (int i = tid; i <= jj; i += kHTThreads) o.T[toff + i] = e(i, jj);
  }
  for (int idx = tid; idx < n * m; idx += kHTThreads) {
    const double x = w(idx / m, n + idx % m);
    o.Bt[idx] = x;
    o.Bt32[idx] = (float)x;
  }
  for (int idx = tid; idx < n * p; idx += kHTThreads) {
    const double x = w(n + idx % p, idx / p);
    o.Ct[idx] = x;
    o.Ct32[idx] = (float)x;
  }
  for (int idx = tid; idx < p * m; idx += kHTThreads) o.D[idx] = in.d(idx / m, idx % m);
}

}  // namespace

size_t reduce_ht_work_bytes(int n, int m, int p) {
  const size_t ldw = (size_t)((n + p) | 1), lde = (size_t)(n | 1);
  return (ldw * (size_t)(n + m) + lde * (size_t)n) * sizeof(double);
}

hipError_t launch_reduce_ht(const ReduceLaunch& L, hipStream_t s) {
  if (L.njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(hess_tri_kernel, dim3(L.njobs), dim3(kHTThreads), 0, s, L);
  return hipGetLastError();
}

}  // namespace lti
