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
//   next pivot column with its norm.  Two barriers per reflector; the steps
//   of one 16-column slot block share straight-line code in which the block
//   index is a compile-time constant, so the slots that v cannot reach are
//   skipped without branches.
// * Global kernel (128 < n <= 256): W (column-major) in a global scratch
//   area that stays hot in L2, three barriers per reflector (build v, left
//   update, right update).  The left update gives each column a group of G
//   adjacent lanes (DPP group sums); the right update gives a wavefront 16
//   consecutive rows and four interleaved quarters of the columns, so that
//   both walk down columns.  Larger models take the blocked reduction
//   (reduce_blocked.hip).
#include <algorithm>
#include <type_traits>

#include "dpp.h"
#include "lti_kernels.h"

// Issue priority of the register reduction's wavefronts (0 = the default of
// the sweep wavefronts that share their CUs, 3 = highest).
#ifndef LTI_REDUCE_PRIO
#define LTI_REDUCE_PRIO 3
#endif

namespace lti {

namespace {

// ---------------------------------------------------------------------------
// Register kernel

constexpr int kRegThreads = 256;

// Sum over the four 16-lane rows of the wavefront (same column position).
__device__ __forceinline__ double sum_thread_rows(double x) { return xor32_sum(xor16_sum(x)); }

template <int T0, int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (T0 < N) {
    f(std::integral_constant<int, T0>{});
    static_for<T0 + 1, N>(f);
  }
}

template <int S>
__global__ __launch_bounds__(kRegThreads) void hess_reg_kernel(const ReduceLaunch L) {
  constexpr int kPad = 16 * S;
  __shared__ double xcol[kPad];  // pivot column kc below row kc, zero elsewhere
  // per wavefront: column sums W^T v (slot blocks 0..S-1) and v^T W v (block S)
  __shared__ double pw[4][kPad + 16];
  __shared__ double ssw[4];  // pivot column sum of squares below row kc+1

  // a reduction is a chain of dependent steps that often shares its CU with
  // sweep wavefronts: let the SIMDs issue its instructions first
  __builtin_amdgcn_s_setprio(LTI_REDUCE_PRIO);
  const ReduceJob job = L.jobs[blockIdx.x];
  const ModelIn in(job);
  const ReducedModel& o = job.out;
  const int n = job.out.n, m = job.out.m, p = job.out.p;
  const int nrow = n + p, ncol = n + m;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int tc = lane & 15;
  const int tr = (wv << 2) | (lane >> 4);
  // slot, within a group of four (two) reduce-scattered values, whose total
  // this lane holds after the exchanges over its wavefront's thread rows
  const int t32 = swap_tag32();
  const int pos4 = 2 * swap_tag16() + t32;

  // Row a of the register block is one vector (kept from the variant with a
  // run-time column slot; every slot index is a compile-time constant now).
  using Row = double __attribute__((ext_vector_type(S < 2 ? 2 : S)));
  Row W[S];
#pragma unroll
  for (int a = 0; a < S; ++a) {
    const int i = tr + 16 * a;
#pragma unroll
    for (int b = 0; b < S; ++b) {
      const int c = tc + 16 * b;
      // the solved system, also kept as given for the extended refinement
      double x = 0.0;
      if (i < n) {
        if (c < n) {
          x = in.a(i, c);
          o.A0[(size_t)c * n + i] = x;
        } else if (c < ncol) {
          x = in.b(i, c - n);
          o.B0[(size_t)(c - n) * n + i] = x;
        }
      } else if (i < nrow && c < n) {
        x = in.c(i - n, c);
        o.C0[(size_t)(i - n) * n + c] = x;
      }
      W[a][b] = x;
    }
  }
  bool live[S];  // this thread's row a is a row of A
#pragma unroll
  for (int a = 0; a < S; ++a) live[a] = tr + 16 * a < n;

  // Publish column kc (its slot block KB = kc / 16 is a compile-time
  // constant): the 16 threads of thread column kc % 16 write every entry of
  // xcol, the column below row kc and zeros elsewhere (so v needs no bounds
  // tests), and the sum of squares below row kc+1.
  auto publish = [&](auto KBc, int kc) {
    constexpr int kb = decltype(KBc)::value;
    const bool mine = tc == (kc & 15);
    double ss = 0.0;
    static_for<0, S>([&](auto A) {
      constexpr int a = decltype(A)::value;
      const int i = tr + 16 * a;
      double x = 0.0;
      // rows of slot blocks below kb lie above kc
      if constexpr (a >= kb) x = (i > kc && live[a]) ? W[a][kb] : 0.0;
      if (mine) xcol[i] = x;
      if constexpr (a == kb || a == kb + 1) x = (i == kc + 1) ? 0.0 : x;
      ss = fma(x, x, ss);
    });
    ss = sum_thread_rows(mine ? ss : 0.0);
    if (lane == (kc & 15)) ssw[wv] = ss;
  };

  if (n > 2) publish(std::integral_constant<int, 0>{}, 0);
  __syncthreads();

  // Steps k = 16 kb .. 16 kb + 15 run the same code with kb a compile-time
  // constant: v vanishes on rows and columns of slot blocks below kb (they lie
  // at or above k), so those products are skipped; the columns of those
  // blocks hold, below the subdiagonal, rounding-level values that are never
  // read again, and are left alone.  Column k is not reset to beta e_{k+1}
  // explicitly: the update itself leaves beta (to rounding) on the
  // subdiagonal and rounding-level values below it.
  static_for<0, S>([&](auto KB) {
    constexpr int kb = decltype(KB)::value;
    const int kend = (16 * kb + 16 < n - 2) ? 16 * kb + 16 : n - 2;
    for (int k = 16 * kb; k < kend; ++k) {
      // reflector of column k, computed by every thread
      double xr[S], xc[S];
#pragma unroll
      for (int a = kb; a < S; ++a) xr[a] = xcol[tr + 16 * a];
#pragma unroll
      for (int b = kb; b < S; ++b) xc[b] = xcol[tc + 16 * b];
      const double ss = (ssw[0] + ssw[1]) + (ssw[2] + ssw[3]);
      const double alpha = xcol[k + 1];
      // branch-free, so that the read of alpha joins the loads above; a
      // column already reduced (ss = 0) takes tau = 0 (P = I)
      const double nrm = sqrt(fma(alpha, alpha, ss));
      const double beta = (alpha >= 0.0) ? -nrm : nrm;
      const bool live = ss != 0.0;
      const double tau = live ? (beta - alpha) / beta : 0.0;
      const double scale = live ? 1.0 / (alpha - beta) : 0.0;
      // v: 1 on row k+1 (slot block kb or kb+1), the scaled column below it
      double vr[S], vc[S];
#pragma unroll
      for (int a = kb; a < S; ++a) {
        vr[a] = xr[a] * scale;
        if (a <= kb + 1) vr[a] = (tr + 16 * a == k + 1) ? 1.0 : vr[a];
      }
#pragma unroll
      for (int b = kb; b < S; ++b) {
        vc[b] = xc[b] * scale;
        if (b <= kb + 1) vc[b] = (tc + 16 * b == k + 1) ? 1.0 : vc[b];
      }
      // keep the reflector (entries below row k+1, and tau)
      if (tc == 0) {
        const int64_t vo = voff(n, k) - (k + 2);
#pragma unroll
        for (int a = kb; a < S; ++a) {
          const int i = tr + 16 * a;
          if (i >= k + 2 && i < n) o.V[vo + i] = vr[a];
        }
        if (tr == 0) o.tau[k] = tau;
      }
      // partial W^T v over this thread's rows, partial W v over its columns
      double pp[S], qq[S];
#pragma unroll
      for (int b = kb; b < S; ++b) {
        pp[b] = 0.0;
#pragma unroll
        for (int a = kb; a < S; ++a) pp[b] = fma(vr[a], W[a][b], pp[b]);
      }
#pragma unroll
      for (int a = 0; a < S; ++a) {
        qq[a] = 0.0;
#pragma unroll
        for (int b = kb; b < S; ++b) qq[a] = fma(W[a][b], vc[b], qq[a]);
        qq[a] = row_sum16_full(qq[a]);  // row sum over the 16 thread columns
      }
      double g = 0.0;
#pragma unroll
      for (int a = kb; a < S; ++a) g = fma(vr[a], qq[a], g);
      // Sums over the wavefront's four thread rows of pp[kb..S-1] and g
      // (value j goes to block kb + j of pw, g to block S): groups of four
      // are reduce-scattered in two swaps, a remaining pair in one swap and
      // one exchange, a remaining single value in two exchanges.
      {
        constexpr int cnt = S - kb + 1;
        double val[cnt];
#pragma unroll
        for (int j = 0; j + 1 < cnt; ++j) val[j] = pp[kb + j];
        val[cnt - 1] = g;
        double* const dst = &pw[wv][tc + 16 * kb];
#pragma unroll
        for (int j = 0; j + 4 <= cnt; j += 4) {
          const double x = rs16_sum(rs32_sum(val[j], val[j + 1]), rs32_sum(val[j + 2], val[j + 3]));
          dst[16 * (j + pos4)] = x;
        }
        constexpr int j2 = cnt & ~3;
        if constexpr ((cnt & 3) >= 2) {
          const double x = xor16_sum(rs32_sum(val[j2], val[j2 + 1]));
          if ((lane & 16) == 0) dst[16 * (j2 + t32)] = x;
        }
        if constexpr ((cnt & 1) == 1) {
          constexpr int j1 = cnt - 1;
          const double x = sum_thread_rows(val[j1]);
          if (lane < 16) dst[16 * j1] = x;
        }
      }
      __syncthreads();

      const double gamma = (pw[0][tc + kPad] + pw[1][tc + kPad]) + (pw[2][tc + kPad] + pw[3][tc + kPad]);
      const double tg = tau * gamma;
#pragma unroll
      for (int b = kb; b < S; ++b) {
        const int c = tc + 16 * b;
        pp[b] = tau * ((pw[0][c] + pw[1][c]) + (pw[2][c] + pw[3][c]));
      }
#pragma unroll
      for (int a = 0; a < S; ++a) qq[a] = tau * (a >= kb ? fma(-tg, vr[a], qq[a]) : qq[a]);
      // W -= v (tau W^T v)^T + tau (q - tau gamma v) v^T
#pragma unroll
      for (int a = 0; a < S; ++a)
#pragma unroll
        for (int b = kb; b < S; ++b) {
          if (a >= kb) W[a][b] = fma(-vr[a], pp[b], W[a][b]);
          W[a][b] = fma(-qq[a], vc[b], W[a][b]);
        }
      if (k + 3 < n) {
        if constexpr (kb + 1 < S) {
          if (((k + 1) & 15) == 0)
            publish(std::integral_constant<int, kb + 1>{}, k + 1);
          else
            publish(KB, k + 1);
        } else {
          publish(KB, k + 1);
        }
      }
      __syncthreads();
    }
  });

  // write the reduced model
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
  for (int idx = threadIdx.x; idx < p * m; idx += kRegThreads) o.D[idx] = in.d(idx / m, idx % m);
}

// ---------------------------------------------------------------------------
// Global kernel

constexpr int kGlobalThreads = 1024;
constexpr int kGlobalGroup = 16;

__host__ __device__ inline int ld_of(int n, int p) { return (n + p) | 1; }

// W column-major in job.work with an odd leading dimension, so that the
// row-strided accesses of the right update spread over the channels.
template <int NT, int G>
__global__ __launch_bounds__(NT) void hess_global_kernel(const ReduceLaunch L) {
  __shared__ double v[kMaxReduceN];
  __shared__ double sc[1];
  const ReduceJob job = L.jobs[blockIdx.x];
  const ModelIn in(job);
  const ReducedModel& o = job.out;
  const int n = job.out.n, m = job.out.m, p = job.out.p;
  const int ldw = ld_of(n, p);
  const int ncol = n + m;
  const int nrow = n + p;
  const int tid = threadIdx.x;
  double* W = job.work;

  for (int idx = tid; idx < nrow * ncol; idx += NT) {
    const int i = idx % nrow;
    const int c = idx / nrow;
    // the solved system, also kept as given for the extended refinement
    double x = 0.0;
    if (i < n) {
      if (c < n) {
        x = in.a(i, c);
        o.A0[(size_t)c * n + i] = x;
      } else {
        x = in.b(i, c - n);
        o.B0[(size_t)(c - n) * n + i] = x;
      }
    } else if (c < n) {
      x = in.c(i - n, c);
      o.C0[(size_t)(i - n) * n + c] = x;
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
      const int64_t vo = voff(n, k) - (k + 2);
      for (int i = k + 2 + tid; i < n; i += 64) {
        const double vi = colk[i] * scale;
        v[i] = vi;
        o.V[vo + i] = vi;
        colk[i] = 0.0;
      }
      if (tid == 0) {
        v[k + 1] = 1.0;
        colk[k + 1] = beta;
        sc[0] = tau;
        o.tau[k] = tau;
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
      // unrolled: several L2 loads in flight per lane instead of one
#pragma unroll 8
      for (int i = k + 1 + lg; i < n; i += G) s = fma(v[i], col[i], s);
      s = group_sum_dpp<G>(s) * tau;
#pragma unroll 8
      for (int i = k + 1 + lg; i < n; i += G) col[i] = fma(-v[i], s, col[i]);
    }
    __syncthreads();

    // right: rows 0..n+p-1 (A and C), columns k+1..n-1.  A wavefront covers
    // 16 consecutive rows (lane % 16) and four interleaved quarters of the
    // columns (lane / 16), so that each load reads 16 consecutive entries of
    // a column (W is column-major); the four partial sums of a row meet
    // through two lane exchanges.
    {
      const int lane = tid & 63, wv = tid >> 6;
      const int lr = lane & 15, q = lane >> 4;
      for (int r0 = 16 * wv; r0 < nrow; r0 += NT / 4) {
        const int r = r0 + lr;
        const bool live = r < nrow;
        double s = 0.0;
        if (live) {
#pragma unroll 8
          for (int c = k + 1 + q; c < n; c += 4) s = fma(W[(size_t)r + (size_t)ldw * c], v[c], s);
        }
        s = xor32_sum(xor16_sum(s)) * tau;
        if (live) {
#pragma unroll 8
          for (int c = k + 1 + q; c < n; c += 4) {
            double* x = W + (size_t)r + (size_t)ldw * c;
            *x = fma(-s, v[c], *x);
          }
        }
      }
    }
    __syncthreads();
  }

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
  for (int idx = tid; idx < p * m; idx += NT) o.D[idx] = in.d(idx / m, idx % m);
}

__global__ __launch_bounds__(256) void zero_kernel(const ZeroLaunch Z) {
  uint32_t* p = Z.e[blockIdx.x].p;
  const uint32_t w = Z.e[blockIdx.x].words;
  for (uint32_t i = threadIdx.x; i < w; i += 256) p[i] = 0u;
}

// One workgroup per finished request: count its point records per path
// code and take the largest estimate (fmaxf skips NaN).
__global__ __launch_bounds__(256) void summarize_kernel(const FinEntry* __restrict__ tab,
                                                        PointSummary* __restrict__ out) {
  __shared__ uint32_t cnt[8];
  __shared__ float mx[4];
  const FinEntry fe = tab[blockIdx.x];
  if (threadIdx.x < 8) cnt[threadIdx.x] = 0u;
  __syncthreads();
  uint32_t c[8] = {0u, 0u, 0u, 0u, 0u, 0u, 0u, 0u};
  float m = 0.0f;
  const uint2* rec = reinterpret_cast<const uint2*>(fe.info);
  for (uint64_t k = threadIdx.x; k < fe.K; k += 256) {
    const uint2 v = rec[k];  // est_rel_err | iters, path, reserved
    const uint32_t path = (v.y >> 8) & 7u;
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) c[q] += (path == q) ? 1u : 0u;
    m = fmaxf(m, __uint_as_float(v.x));
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    uint32_t x = c[q];
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    if ((threadIdx.x & 63) == 0 && x) atomicAdd(&cnt[q], x);
  }
  for (int o = 32; o >= 1; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) mx[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    PointSummary s{};
    for (int q = 0; q < 8; ++q) s.count[q] = cnt[q];
    s.max_est = fmaxf(fmaxf(mx[0], mx[1]), fmaxf(mx[2], mx[3]));
    out[blockIdx.x] = s;
  }
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

size_t reduced_bytes(int n, int m, int p, bool desc) {
  const size_t hl = (size_t)hlen(n);
  return align256(hl * 8) + align256((size_t)n * m * 8) + align256((size_t)n * p * 8) +
         align256((size_t)p * m * 8) + align256(hl * 4) + align256((size_t)n * m * 4) +
         align256((size_t)n * p * 4) + align256((size_t)n * n * 8) + align256((size_t)n * m * 8) +
         align256((size_t)p * n * 8) + align256((size_t)vlen(n) * 8) + align256((size_t)n * 8) +
         (desc ? align256((size_t)n * (n + 1) / 2 * 8) : 0);
}

void reduced_layout(void* base, int n, int m, int p, int trans, ReducedModel* o, bool desc) {
  char* b = static_cast<char*>(base);
  const size_t hl = (size_t)hlen(n);
  auto take = [&b](size_t bytes) {
    char* x = b;
    b += align256(bytes);
    return x;
  };
  o->H = reinterpret_cast<double*>(take(hl * 8));
  o->Bt = reinterpret_cast<double*>(take((size_t)n * m * 8));
  o->Ct = reinterpret_cast<double*>(take((size_t)n * p * 8));
  o->D = reinterpret_cast<double*>(take((size_t)p * m * 8));
  o->H32 = reinterpret_cast<float*>(take(hl * 4));
  o->Bt32 = reinterpret_cast<float*>(take((size_t)n * m * 4));
  o->Ct32 = reinterpret_cast<float*>(take((size_t)n * p * 4));
  o->A0 = reinterpret_cast<double*>(take((size_t)n * n * 8));
  o->B0 = reinterpret_cast<double*>(take((size_t)n * m * 8));
  o->C0 = reinterpret_cast<double*>(take((size_t)p * n * 8));
  o->V = reinterpret_cast<double*>(take((size_t)vlen(n) * 8));
  o->tau = reinterpret_cast<double*>(take((size_t)n * 8));
  o->T = desc ? reinterpret_cast<double*>(take((size_t)n * (n + 1) / 2 * 8)) : nullptr;
  o->n = n;
  o->m = m;
  o->p = p;
  o->trans = trans;
}

hipError_t launch_zero(const ZeroLaunch& Z, hipStream_t s) {
  if (Z.n <= 0) return hipSuccess;
  if (Z.n > kMaxZero) return hipErrorInvalidValue;
  zero_kernel<<<Z.n, 256, 0, s>>>(Z);
  return hipGetLastError();
}

hipError_t launch_summarize(const FinEntry* tab, PointSummary* out, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  summarize_kernel<<<n, 256, 0, s>>>(tab, out);
  return hipGetLastError();
}

hipError_t launch_reduce(const ReduceLaunch& L, int rclass, hipStream_t s) {
  if (L.njobs <= 0) return hipSuccess;
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
    case kReduceHT:
      return launch_reduce_ht(L, s);
    case kReduceBlocked:
      return launch_reduce_blocked(L.host_jobs, L.njobs, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace lti
