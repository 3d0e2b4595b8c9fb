// Householder reduction to upper Hessenberg form, one workgroup per model.
//
// For k = 0 .. n-3 a reflector P_k = I - tau v v^T (v[k+1] = 1, LAPACK
// dlarfg sign convention: P_k x = beta e_1, beta = -sign(x_1) ||x||)
// annihilates column k below the subdiagonal, and is applied from the left
// to rows k+1..n-1 of [A | B] and from the right to columns k+1..n-1 of
// [A ; C] (Golub & Van Loan, Matrix Computations, 4th ed., Algorithm 7.4.2).
// At the end the working matrix holds H = Q^T A Q, Q^T B and C Q.
//
// The augmented (n+p) x (n+m) working matrix W = [[A, B], [C, *]] lives in
// LDS when it fits (n <= 128 with m, p <= 8 does: at most 149 KB of the
// 160 KB per CU), otherwise in a global scratch area that stays hot in L2.
// W is column-major with an odd leading dimension so that the row-strided
// accesses of the right update spread over the LDS banks.
//
// Every reflector costs three workgroup barriers: build v (wave 0, DPP wave
// sum of squares), left update (a group of G adjacent lanes per column:
// partial dot products over Q interleaved rows, a DPP sum within the group,
// then the rank-1 update of the same column), right update (a group of G
// lanes per row, likewise).  The Q-element inner loops are unrolled and
// predicated so that their LDS loads issue back to back.
#include "dpp.h"
#include "lti_kernels.h"

namespace lti {

namespace {

__host__ __device__ inline int ld_of(int n, int p) { return (n + p) | 1; }

template <int NT, int G, int Q, bool kLds>
__global__ __launch_bounds__(NT) void hess_kernel(const ReduceJob* __restrict__ jobs) {
  extern __shared__ double smem[];
  const ReduceJob job = jobs[blockIdx.x];
  const int n = job.out.n, m = job.out.m, p = job.out.p;
  const int ldw = ld_of(n, p);
  const int ncol = n + m;
  const int nrow = n + p;
  const int tid = threadIdx.x;
  double* W;
  double* v;
  double* sc;
  if (kLds) {
    W = smem;
    v = smem + (size_t)ldw * ncol;
  } else {
    W = job.work;
    v = smem;
  }
  sc = v + n;

  // load [[A, B], [C, *]] column-major
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
    if constexpr (Q == 0) {
      for (int c = k + 1 + group; c < ncol; c += kGroups) {
        double* col = W + (size_t)ldw * c;
        double s = 0.0;
        for (int i = k + 1 + lg; i < n; i += G) s = fma(v[i], col[i], s);
        s = group_sum_dpp<G>(s) * tau;
        for (int i = k + 1 + lg; i < n; i += G) col[i] = fma(-v[i], s, col[i]);
      }
    } else {
      double vv[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int i = k + 1 + lg + G * q;
        vv[q] = (i < n) ? v[i] : 0.0;
      }
      for (int c = k + 1 + group; c < ncol; c += kGroups) {
        double* col = W + (size_t)ldw * c;
        double xx[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int i = k + 1 + lg + G * q;
          xx[q] = (i < n) ? col[i] : 0.0;
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) s = fma(vv[q], xx[q], s);
        s = group_sum_dpp<G>(s) * tau;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int i = k + 1 + lg + G * q;
          if (i < n) col[i] = fma(-vv[q], s, xx[q]);
        }
      }
    }
    __syncthreads();

    // right: rows 0..n+p-1 (A and C), columns k+1..n-1
    if constexpr (Q == 0) {
      for (int r = group; r < nrow; r += kGroups) {
        double s = 0.0;
        for (int c = k + 1 + lg; c < n; c += G) s = fma(W[(size_t)r + (size_t)ldw * c], v[c], s);
        s = group_sum_dpp<G>(s) * tau;
        for (int c = k + 1 + lg; c < n; c += G) {
          double* x = W + (size_t)r + (size_t)ldw * c;
          *x = fma(-s, v[c], *x);
        }
      }
    } else {
      double vv[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int c = k + 1 + lg + G * q;
        vv[q] = (c < n) ? v[c] : 0.0;
      }
      for (int r = group; r < nrow; r += kGroups) {
        double xx[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = k + 1 + lg + G * q;
          xx[q] = (c < n) ? W[(size_t)r + (size_t)ldw * c] : 0.0;
        }
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q) s = fma(xx[q], vv[q], s);
        s = group_sum_dpp<G>(s) * tau;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          const int c = k + 1 + lg + G * q;
          if (c < n) W[(size_t)r + (size_t)ldw * c] = fma(-s, vv[q], xx[q]);
        }
      }
    }
    __syncthreads();
  }

  // write the reduced model
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

// LDS kernel: 1024 threads; a column (row) is shared by G lanes holding Q
// interleaved rows (columns) each: G = 16 up to 64 states, 8 up to 128.
constexpr int kLdsThreads = 1024;
constexpr int kGlobalThreads = 1024;
constexpr int kGlobalGroup = 8;
constexpr size_t kLdsLimit = 160 * 1024;

size_t lds_bytes(int n, int m, int p) {
  return ((size_t)ld_of(n, p) * (size_t)(n + m) + (size_t)n + 8) * sizeof(double);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

using ReduceFn = void (*)(const ReduceJob*);

template <int G, int Q>
hipError_t launch_lds(const ReduceJob* jobs, int njobs, size_t lds_need, hipStream_t s) {
  static bool attr_set = false;  // launches come from one scheduler thread
  const void* fn = reinterpret_cast<const void*>(&hess_kernel<kLdsThreads, G, Q, true>);
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsLimit);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hess_kernel<kLdsThreads, G, Q, true><<<njobs, kLdsThreads, lds_need, s>>>(jobs);
  return hipGetLastError();
}

}  // namespace

bool reduce_fits_lds(int n, int m, int p) { return lds_bytes(n, m, p) <= kLdsLimit; }

size_t reduce_lds_bytes(int n, int m, int p) { return lds_bytes(n, m, p); }

int reduce_class(int n, int m, int p) {
  if (!reduce_fits_lds(n, m, p) || n > 128) return kReduceGlobal;
  return (n <= 16) ? 0 : (n <= 32) ? 1 : (n <= 64) ? 2 : 3;
}

size_t reduce_work_bytes(int n, int m, int p) {
  if (reduce_class(n, m, p) != kReduceGlobal) return 0;
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

hipError_t launch_reduce(const ReduceJob* jobs, int njobs, int rclass, size_t lds_need, hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  if (rclass == kReduceGlobal) {
    // v (n <= kMaxReduceN doubles) plus scalars
    const size_t sh = (kMaxReduceN + 8) * sizeof(double);
    hess_kernel<kGlobalThreads, kGlobalGroup, 0, false><<<njobs, kGlobalThreads, sh, s>>>(jobs);
    return hipGetLastError();
  }
  if (lds_need > kLdsLimit) return hipErrorInvalidValue;
  switch (rclass) {
    case 0: return launch_lds<16, 1>(jobs, njobs, lds_need, s);
    case 1: return launch_lds<16, 2>(jobs, njobs, lds_need, s);
    case 2: return launch_lds<16, 4>(jobs, njobs, lds_need, s);
    case 3: return launch_lds<8, 16>(jobs, njobs, lds_need, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lti
