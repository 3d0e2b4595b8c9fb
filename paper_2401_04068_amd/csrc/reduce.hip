// Householder reduction to upper Hessenberg form, one workgroup per model.
//
// For k = 0 .. n-3 a reflector P_k = I - tau v v^T (v[k+1] = 1, LAPACK
// dlarfg sign convention: P_k x = beta e_1, beta = -sign(x_1) ||x||)
// annihilates column k below the subdiagonal, and is applied from the left
// to rows k+1..n-1 of [A | B] and from the right to columns k+1..n-1 of
// [A ; C] (Golub & Van Loan, Matrix Computations, 4th ed., Algorithm 7.4.2).
// At the end the working matrix holds H = Q^T A Q, Q^T B and C Q.
//
// Two kernels work on the augmented (n+p) x (n+m) matrix W = [[A, B], [C, *]]:
//
// * Register kernel (n <= 128).  256 threads form a 16 x 16 grid; thread
//   (r, c) holds W(i, j) for i = r (mod 16), j = c (mod 16) in an S x S
//   register array, S = ceil(max(n+p, n+m) / 16).  The two one-sided updates
//   of a step are applied together as one rank-2 update computed from the old
//   matrix,
//       P W P = W - v (tau W^T v)^T - tau (q - tau gamma v) v^T,
//       q = W v,  gamma = v^T W v,
//   so a step needs two exchanges: the row sums q (a DPP sum inside each
//   16-lane row) with the column sums W^T v (over the 16 thread rows: two
//   lane shuffles inside the wavefront, then LDS across the four), and the
//   next pivot column with its norm.  Two barriers per reflector; the step
//   is straight-line code over all S x S slots.
// * Global kernel (128 < n <= 256): W in a global scratch area that stays
//   hot in L2, three barriers per reflector (build v, left update, right
//   update), a group of G adjacent lanes per column or row with DPP group
//   sums.  Larger models take the blocked reduction (reduce_blocked.hip).
#include <algorithm>

#include "dpp.h"
#include "lti_kernels.h"

namespace lti {

namespace {

// ---------------------------------------------------------------------------
// Register kernel

constexpr int kRegThreads = 256;

// Sum over the four 16-lane rows of the wavefront (same column position).
__device__ __forceinline__ double sum_thread_rows(double x) { return xor32_sum(xor16_sum(x)); }

template <int S>
__global__ __launch_bounds__(kRegThreads) void hess_reg_kernel(const ReduceLaunch L) {
  constexpr int kPad = 16 * S;
  __shared__ double xcol[kPad];   // pivot column, rows k+1 .. n-1
  __shared__ double pw[4][kPad];  // column sums W^T v, one partial per wavefront
  __shared__ double ssw[4];       // pivot column sum of squares below row k+1
  __shared__ double gw[4];        // v^T W v partials

  // a reduction is a chain of dependent steps that often shares its CU with
  // sweep wavefronts: let the SIMDs issue its instructions first
  __builtin_amdgcn_s_setprio(3);
  const ReduceJob job = L.job[blockIdx.x];
  const int n = job.out.n, m = job.out.m, p = job.out.p;
  const int nrow = n + p, ncol = n + m;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int tc = lane & 15;
  const int tr = (wv << 2) | (lane >> 4);

  // Row a of the register block is one vector, so that reading the column
  // slot kb (uniform, known at run time) is an indexed register move, not a
  // trip through scratch memory.
  using Row = double __attribute__((ext_vector_type(S < 2 ? 2 : S)));
  Row W[S];
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int i = tr + 16 * a;
#pragma unroll
    for (int b = 0; b < S; ++b) {
      const int c = tc + 16 * b;
      double x = 0.0;
      if (i < n) {
        if (c < n)
          x = job.A[(size_t)i * n + c];
        else if (c < ncol)
          x = job.B[(size_t)i * m + (c - n)];
      } else if (i < nrow && c < n) {
        x = job.C[(size_t)(i - n) * n + c];
      }
      W[a][b] = x;
    }
  }

  // Publish column kc (rows kc+1 .. n-1) and its sum of squares below row
  // kc+1; only the 16 threads of thread column kc % 16 hold it.
  auto publish = [&](int kc) {
    const int kb = kc >> 4;
    const bool mine = tc == (kc & 15);
    double x[S];
#pragma unroll
    for (int a = 0; a < S; ++a) x[a] = W[a][kb];
    double ss = 0.0;
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const int i = tr + 16 * a;
      if (mine && i > kc && i < n) xcol[i] = x[a];
      const double x2 = (i > kc + 1 && i < n) ? x[a] : 0.0;
      ss = fma(x2, x2, ss);
    }
    ss = sum_thread_rows(mine ? ss : 0.0);
    if (lane == (kc & 15)) ssw[wv] = ss;
  };

  if (n > 2) publish(0);
  __syncthreads();

  // Every step runs the same straight-line code over all S x S slots: slots
  // outside the active rows and columns meet exact zeros of v (a taken branch
  // costs more than the few fused multiply-adds it would skip).  Column k is
  // not reset to beta e_{k+1} explicitly: the update itself leaves beta (to
  // rounding) on the subdiagonal and rounding-level values below it, which
  // are never read again (H is stored up to the subdiagonal, and later
  // reflectors only touch those rows through their own rounding-level
  // column sums).
  for (int k = 0; k + 2 < n; ++k) {
    // reflector of column k, computed by every thread
    double xr[S], xc[S];
#pragma unroll
    for (int a = 0; a < S; ++a) xr[a] = xcol[tr + 16 * a];
#pragma unroll
    for (int b = 0; b < S; ++b) xc[b] = xcol[tc + 16 * b];
    const double ss = (ssw[0] + ssw[1]) + (ssw[2] + ssw[3]);
    const double alpha = xcol[k + 1];
    double tau = 0.0, scale = 0.0;
    if (ss != 0.0) {
      const double nrm = sqrt(fma(alpha, alpha, ss));
      const double beta = (alpha >= 0.0) ? -nrm : nrm;
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    // v on this thread's rows and columns (stale or unwritten entries of
    // xcol are never selected)
    double vr[S], vc[S];
#pragma unroll
    for (int a = 0; a < S; ++a) {
      const int i = tr + 16 * a;
      const double t = xr[a] * scale;
      vr[a] = (i == k + 1) ? 1.0 : ((i > k + 1 && i < n) ? t : 0.0);
    }
#pragma unroll
    for (int b = 0; b < S; ++b) {
      const int c = tc + 16 * b;
      const double t = xc[b] * scale;
      vc[b] = (c == k + 1) ? 1.0 : ((c > k + 1 && c < n) ? t : 0.0);
    }
    // partial W^T v over this thread's rows, partial W v over its columns
    double pp[S], qq[S];
#pragma unroll
    for (int b = 0; b < S; ++b) {
      pp[b] = 0.0;
#pragma unroll
      for (int a = 0; a < S; ++a) pp[b] = fma(vr[a], W[a][b], pp[b]);
    }
#pragma unroll
    for (int a = 0; a < S; ++a) {
      qq[a] = 0.0;
#pragma unroll
      for (int b = 0; b < S; ++b) qq[a] = fma(W[a][b], vc[b], qq[a]);
      qq[a] = group_sum_dpp<16>(qq[a]);  // row sum over the 16 thread columns
    }
    double g = 0.0;
#pragma unroll
    for (int a = 0; a < S; ++a) g = fma(vr[a], qq[a], g);
    g = sum_thread_rows(g);
#pragma unroll
    for (int b = 0; b < S; ++b) {
      pp[b] = sum_thread_rows(pp[b]);
      if (lane < 16) pw[wv][tc + 16 * b] = pp[b];
    }
    if (lane == 0) gw[wv] = g;
    __syncthreads();

    double pr[4][S];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int b = 0; b < S; ++b) pr[w][b] = pw[w][tc + 16 * b];
    const double gamma = (gw[0] + gw[1]) + (gw[2] + gw[3]);
    const double tg = tau * gamma;
#pragma unroll
    for (int b = 0; b < S; ++b) pp[b] = tau * ((pr[0][b] + pr[1][b]) + (pr[2][b] + pr[3][b]));
#pragma unroll
    for (int a = 0; a < S; ++a) qq[a] = tau * fma(-tg, vr[a], qq[a]);
    // W -= v (tau W^T v)^T + tau (q - tau gamma v) v^T
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; b < S; ++b) {
        W[a][b] = fma(-vr[a], pp[b], W[a][b]);
        W[a][b] = fma(-qq[a], vc[b], W[a][b]);
      }
    if (k + 3 < n) publish(k + 1);
    __syncthreads();
  }

  // write the reduced model
  const ReducedModel& o = job.out;
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int i = tr + 16 * a;
#pragma unroll
    for (int b = 0; b < S; ++b) {
      const int c = tc + 16 * b;
      const double x = W[a][b];
      if (i < n) {
        if (c < n) {
          if (i <= c + 1) {
            const int64_t off = hoff(c) + i;
            o.H[off] = x;
            o.H32[off] = (float)x;
          }
        } else if (c < ncol) {
          const int idx = i * m + (c - n);
          o.Bt[idx] = x;
          o.Bt32[idx] = (float)x;
        }
      } else if (i < nrow && c < n) {
        const int idx = c * p + (i - n);
        o.Ct[idx] = x;
        o.Ct32[idx] = (float)x;
      }
    }
  }
  for (int idx = threadIdx.x; idx < p * m; idx += kRegThreads) o.D[idx] = job.D ? job.D[idx] : 0.0;
}

// ---------------------------------------------------------------------------
// Global kernel

constexpr int kGlobalThreads = 1024;
constexpr int kGlobalGroup = 8;

__host__ __device__ inline int ld_of(int n, int p) { return (n + p) | 1; }

// W column-major in job.work with an odd leading dimension, so that the
// row-strided accesses of the right update spread over the channels.
template <int NT, int G>
__global__ __launch_bounds__(NT) void hess_global_kernel(const ReduceLaunch L) {
  __shared__ double v[kMaxReduceN];
  __shared__ double sc[1];
  const ReduceJob job = L.job[blockIdx.x];
  const int n = job.out.n, m = job.out.m, p = job.out.p;
  const int ldw = ld_of(n, p);
  const int ncol = n + m;
  const int nrow = n + p;
  const int tid = threadIdx.x;
  double* W = job.work;

  for (int idx = tid; idx < nrow * ncol; idx += NT) {
    const int i = idx % nrow;
    const int c = idx / nrow;
    double x = 0.0;
    if (i < n) {
      x = (c < n) ? job.A[(size_t)i * n + c] : job.B[(size_t)i * m + (c - n)];
    } else if (c < n) {
      x = job.C[(size_t)(i - n) * n + c];
    }
    W[(size_t)i + (size_t)ldw * c] = x;
  }
  __syncthreads();

  const int lg = tid & (G - 1);
  const int group = tid / G;
  constexpr int kGroups = NT / G;

  for (int k = 0; k + 2 < n; ++k) {
    double* colk = W + (size_t)ldw * k;
    if (tid < 64) {
      const double alpha = colk[k + 1];
      double ss = 0.0;
      for (int i = k + 2 + tid; i < n; i += 64) {
        const double x = colk[i];
        ss = fma(x, x, ss);
      }
      ss = wave_sum_dpp(ss);
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (ss != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, ss));
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      for (int i = k + 2 + tid; i < n; i += 64) {
        v[i] = colk[i] * scale;
        colk[i] = 0.0;
      }
      if (tid == 0) {
        v[k + 1] = 1.0;
        colk[k + 1] = beta;
        sc[0] = tau;
      }
    }
    __syncthreads();
    // tau == 0 (column already reduced) makes both updates exact no-ops; they
    // still run so that every wave passes the same barriers.
    const double tau = sc[0];

    // left: rows k+1..n-1, columns k+1..n+m-1 (A and B)
    for (int c = k + 1 + group; c < ncol; c += kGroups) {
      double* col = W + (size_t)ldw * c;
      double s = 0.0;
      for (int i = k + 1 + lg; i < n; i += G) s = fma(v[i], col[i], s);
      s = group_sum_dpp<G>(s) * tau;
      for (int i = k + 1 + lg; i < n; i += G) col[i] = fma(-v[i], s, col[i]);
    }
    __syncthreads();

    // right: rows 0..n+p-1 (A and C), columns k+1..n-1
    for (int r = group; r < nrow; r += kGroups) {
      double s = 0.0;
      for (int c = k + 1 + lg; c < n; c += G) s = fma(W[(size_t)r + (size_t)ldw * c], v[c], s);
      s = group_sum_dpp<G>(s) * tau;
      for (int c = k + 1 + lg; c < n; c += G) {
        double* x = W + (size_t)r + (size_t)ldw * c;
        *x = fma(-s, v[c], *x);
      }
    }
    __syncthreads();
  }

  const ReducedModel& o = job.out;
  for (int j = 0; j < n; ++j) {
    const int len = (j + 2 < n) ? j + 2 : n;
    const int64_t off = hoff(j);
    for (int i = tid; i < len; i += NT) {
      const double x = W[(size_t)i + (size_t)ldw * j];
      o.H[off + i] = x;
      o.H32[off + i] = (float)x;
    }
  }
  for (int idx = tid; idx < n * m; idx += NT) {
    const int i = idx / m, j = idx % m;
    const double x = W[(size_t)i + (size_t)ldw * (n + j)];
    o.Bt[idx] = x;
    o.Bt32[idx] = (float)x;
  }
  for (int idx = tid; idx < n * p; idx += NT) {
    const int i = idx / p, a = idx % p;
    const double x = W[(size_t)(n + a) + (size_t)ldw * i];
    o.Ct[idx] = x;
    o.Ct32[idx] = (float)x;
  }
  for (int idx = tid; idx < p * m; idx += NT) o.D[idx] = job.D ? job.D[idx] : 0.0;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <int S>
hipError_t launch_reg(const ReduceLaunch& L, hipStream_t s) {
  hess_reg_kernel<S><<<L.njobs, kRegThreads, 0, s>>>(L);
  return hipGetLastError();
}

}  // namespace

int reduce_class(int n, int m, int p) {
  const int s = (std::max(n + p, n + m) + 15) / 16;
  if (n <= kMaxRegReduceN && s <= kNumRegClasses) return s - 1;
  return n <= kMaxGlobalReduceN ? kReduceGlobal : kReduceBlocked;
}

size_t reduce_work_bytes(int n, int m, int p) {
  const int rc = reduce_class(n, m, p);
  if (rc == kReduceBlocked) return align256(reduce_blocked_work_bytes(n, m, p));
  if (rc != kReduceGlobal) return 0;
  return align256((size_t)ld_of(n, p) * (size_t)(n + m) * sizeof(double));
}

size_t reduced_bytes(int n, int m, int p) {
  const size_t hl = (size_t)hlen(n);
  return align256(hl * 8) + align256((size_t)n * m * 8) + align256((size_t)n * p * 8) +
         align256((size_t)p * m * 8) + align256(hl * 4) + align256((size_t)n * m * 4) +
         align256((size_t)n * p * 4);
}

void reduced_layout(void* base, int n, int m, int p, ReducedModel* o) {
  char* b = static_cast<char*>(base);
  const size_t hl = (size_t)hlen(n);
  o->H = reinterpret_cast<double*>(b);
  b += align256(hl * 8);
  o->Bt = reinterpret_cast<double*>(b);
  b += align256((size_t)n * m * 8);
  o->Ct = reinterpret_cast<double*>(b);
  b += align256((size_t)n * p * 8);
  o->D = reinterpret_cast<double*>(b);
  b += align256((size_t)p * m * 8);
  o->H32 = reinterpret_cast<float*>(b);
  b += align256(hl * 4);
  o->Bt32 = reinterpret_cast<float*>(b);
  b += align256((size_t)n * m * 4);
  o->Ct32 = reinterpret_cast<float*>(b);
  o->n = n;
  o->m = m;
  o->p = p;
  o->pad = 0;
}

hipError_t launch_reduce(const ReduceLaunch& L, int rclass, hipStream_t s) {
  if (L.njobs <= 0) return hipSuccess;
  if (L.njobs > kMaxInlineJobs) return hipErrorInvalidValue;
  switch (rclass) {
    case 0: return launch_reg<1>(L, s);
    case 1: return launch_reg<2>(L, s);
    case 2: return launch_reg<3>(L, s);
    case 3: return launch_reg<4>(L, s);
    case 4: return launch_reg<5>(L, s);
    case 5: return launch_reg<6>(L, s);
    case 6: return launch_reg<7>(L, s);
    case 7: return launch_reg<8>(L, s);
    case 8: return launch_reg<9>(L, s);
    case kReduceGlobal:
      hess_global_kernel<kGlobalThreads, kGlobalGroup><<<L.njobs, kGlobalThreads, 0, s>>>(L);
      return hipGetLastError();
    case kReduceBlocked:
      for (int i = 0; i < L.njobs; ++i) {
        const hipError_t e = launch_reduce_blocked(L.job[i], s);
        if (e != hipSuccess) return e;
      }
      return hipSuccess;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lti
