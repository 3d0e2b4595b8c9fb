// Robust value iteration for interval MDPs (the paper's Eq. 2, inner problem
// Eq. 3 by O-maximization, section 4), one MI355X.
//
// One wavefront per state and iteration: for each of the state's columns
// (state-action pairs) the wave loads the column's destinations (coalesced
// rowval / lower / gap, V gathered through L2, where the whole value vector
// of a large model stays), computes
//
//   value = sum lower V + sum_{o before t} gap_o V_o + (rem - sum_{o before t} gap_o) V_t
//
// where rem = 1 - sum lower and t is the threshold destination of the
// O-maximization ordering (ascending V for a minimising adversary,
// descending for a maximising one): the first destination at which the
// gaps handed out in that order reach rem.  That is the same distribution
// the sequential procedure builds, and the same value, without sorting: the
// ordering matters only through t.
//
// Finding t: destinations are compared by 64-bit keys that order like their
// values (the IEEE bit pattern with the sign handled; complemented for the
// descending order).  The column remembers the position of last iteration's
// threshold; its current value is tested first with one fused pass of wave
// sums (gaps strictly before it, gaps up to it).  Rankings change little
// between iterations, so that test usually settles t.  Otherwise a
// bisection over the keys narrows the candidate range: each round takes the
// smallest and largest candidate key (wave min / max) and splits at the
// highest bit in which they differ, keeping the half in which the gaps reach
// rem; the highest differing bit drops every round, so at most 64 rounds.
// Every wave reduction is an all-lanes butterfly (DPP within rows, gfx950
// permlane swaps across rows), so every lane holds the bitwise-same result.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "dpp.h"
#include "imdp_vi.h"

namespace imdp {
namespace {

using lti::dpp_full;
using lti::kDppQuadSwap1;
using lti::kDppQuadSwap2;
using lti::kDppRowHalfMirror;
using lti::kDppRowMirror;

constexpr int kWavesPerBlock = 4;
constexpr int kThreads = 64 * kWavesPerBlock;

// ------------------------------------------------------------ wave reductions
// All 64 lanes must be active.

__device__ __forceinline__ double wsum(double x) {
  x += dpp_full<kDppQuadSwap1>(x);
  x += dpp_full<kDppQuadSwap2>(x);
  x += dpp_full<kDppRowHalfMirror>(x);
  x += dpp_full<kDppRowMirror>(x);
  x = lti::xor16_sum(x);
  return lti::xor32_sum(x);
}

template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x) {
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)x, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(x >> 32), CTRL, 0xf, 0xf, false);
  return ((uint64_t)hi << 32) | lo;
}

// (x[l], x[l ^ 16]) and (x[l], x[l ^ 32]) through the permlane swaps.
__device__ __forceinline__ void swap16_u64(uint64_t x, uint64_t& a, uint64_t& b) {
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)x, (unsigned)x, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(x >> 32), (unsigned)(x >> 32), false, false);
  a = ((uint64_t)h[0] << 32) | l[0];
  b = ((uint64_t)h[1] << 32) | l[1];
}
__device__ __forceinline__ void swap32_u64(uint64_t x, uint64_t& a, uint64_t& b) {
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)x, (unsigned)x, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(x >> 32), (unsigned)(x >> 32), false, false);
  a = ((uint64_t)h[0] << 32) | l[0];
  b = ((uint64_t)h[1] << 32) | l[1];
}

__device__ __forceinline__ uint64_t wmin(uint64_t x) {
  uint64_t y = dpp_u64<kDppQuadSwap1>(x);
  x = y < x ? y : x;
  y = dpp_u64<kDppQuadSwap2>(x);
  x = y < x ? y : x;
  y = dpp_u64<kDppRowHalfMirror>(x);
  x = y < x ? y : x;
  y = dpp_u64<kDppRowMirror>(x);
  x = y < x ? y : x;
  uint64_t a, b;
  swap16_u64(x, a, b);
  x = a < b ? a : b;
  swap32_u64(x, a, b);
  return a < b ? a : b;
}

__device__ __forceinline__ uint64_t wmax(uint64_t x) {
  uint64_t y = dpp_u64<kDppQuadSwap1>(x);
  x = y > x ? y : x;
  y = dpp_u64<kDppQuadSwap2>(x);
  x = y > x ? y : x;
  y = dpp_u64<kDppRowHalfMirror>(x);
  x = y > x ? y : x;
  y = dpp_u64<kDppRowMirror>(x);
  x = y > x ? y : x;
  uint64_t a, b;
  swap16_u64(x, a, b);
  x = a > b ? a : b;
  swap32_u64(x, a, b);
  return a > b ? a : b;
}

// ------------------------------------------------------------ keys

// Unsigned key that orders like the double (finite values).
__device__ __forceinline__ uint64_t key_of(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double value_of(uint64_t k) {
  const uint64_t b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}
// Order key: ascending values for a minimising adversary, descending for a
// maximising one.
__device__ __forceinline__ uint64_t okey(double v, bool pess) {
  const uint64_t k = key_of(v);
  return pess ? k : ~k;
}
__device__ __forceinline__ double ovalue(uint64_t k, bool pess) { return value_of(pess ? k : ~k); }

// ------------------------------------------------------------ model

struct Dev {
  const int* stateptr;
  const int* colptr;
  const int* rowval;
  const double* lower;
  const double* gap;
  const double* rem;   // per column: 1 - sum lower
  const double* gtot;  // per column: sum of gaps
  int* tpos;           // per column: position of the last threshold
};

struct StepArgs {
  Dev d;
  const double* Vin;
  double* Vout;
  const double* fixed;   // NaN: updated by the recursion; else the held value
  const double* reward;  // reward property: r(s), else null
  double discount;
  int* policy;           // null, or the slot of this iteration: policy[s * stride]
  int policy_stride;
  double* partial;       // null, or per-block max |V_k - V_{k-1}|
  const int* states;     // the states of this launch (one column class)
  int n_list;
  int pessimistic;
  int maximize;
};

// The elements of one column as R register chunks of 64 (m <= 64 R).
template <int R>
struct RegCol {
  double v[R], g[R];
  int m;
  template <typename F>
  __device__ __forceinline__ void each(F f) const {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < R; ++r) f(v[r], g[r], lane + 64 * r < m, lane + 64 * r);
  }
};

// The elements of a long column, reloaded from memory on every pass.
struct StreamCol {
  const int* rv;
  const double* gp;
  const double* V;
  int m;
  template <typename F>
  __device__ __forceinline__ void each(F f) const {
    const int lane = threadIdx.x & 63;
    for (int c = 0; c < m; c += 64) {
      const int i = c + lane;
      const bool ok = i < m;
      const double v = ok ? V[rv[i]] : 0.0;
      const double g = ok ? gp[i] : 0.0;
      f(v, g, ok, i);
    }
  }
};

// Threshold search and value once the elements and base = sum lower V are
// known (base already summed over the wave).
template <typename Col>
__device__ __forceinline__ double col_finish(const Dev& d, int j, int a, const Col& col, const double* V, double base,
                                             bool pess) {
  const int lane = threadIdx.x & 63;
  const int m = col.m;
  const double rem = d.rem[j];
  if (!(rem > 0.0)) return base;  // the lower bounds already carry all the mass
  if (d.gtot[j] <= rem) {         // every gap is handed out
    double s = 0.0;
    col.each([&](double v, double g, bool ok, int) {
      if (ok) s = fma(g, v, s);
    });
    return base + wsum(s);
  }
  // warm start: the threshold position of the previous iteration
  int tp = d.tpos[j];
  if (tp < 0 || tp >= m) tp = 0;
  const double vt = V[d.rowval[a + tp]];
  const uint64_t kt = okey(vt, pess);
  double lt = 0.0, le = 0.0, vgl = 0.0;
  col.each([&](double v, double g, bool ok, int) {
    const uint64_t k = okey(v, pess);
    if (ok && k < kt) {
      lt += g;
      vgl = fma(g, v, vgl);
    }
    if (ok && k <= kt) le += g;
  });
  lt = wsum(lt);
  le = wsum(le);
  vgl = wsum(vgl);
  if (lt < rem && rem <= le) return base + vgl + (rem - lt) * vt;

  // bisection over the candidate keys [lo, hi]: invariant
  // sum_{key < lo} gap < rem <= sum_{key <= hi} gap
  uint64_t lo, hi;
  if (le < rem) {
    lo = kt + 1;
    hi = ~0ull;
  } else {
    lo = 0;
    hi = kt - 1;  // lt >= rem > 0: some key is below kt
  }
  uint64_t kstar = lo;
  for (int round = 0; round < 70; ++round) {
    uint64_t cmin = ~0ull, cmax = 0;
    col.each([&](double v, double, bool ok, int) {
      const uint64_t k = okey(v, pess);
      if (ok && k >= lo && k <= hi) {
        cmin = k < cmin ? k : cmin;
        cmax = k > cmax ? k : cmax;
      }
    });
    cmin = wmin(cmin);
    cmax = wmax(cmax);
    kstar = cmin;
    if (cmin >= cmax) break;  // one distinct key left
    const int b = 63 - __builtin_clzll(cmin ^ cmax);
    const uint64_t mid = (cmax >> b) << b;  // cmin < mid <= cmax
    double s = 0.0;
    col.each([&](double v, double g, bool ok, int) {
      if (ok && okey(v, pess) < mid) s += g;
    });
    s = wsum(s);
    if (s >= rem)
      hi = mid - 1;
    else
      lo = mid;
  }
  // sums below the threshold, and the threshold's first position for the
  // next iteration
  lt = 0.0;
  vgl = 0.0;
  int pos = 0x7fffffff;
  col.each([&](double v, double g, bool ok, int i) {
    const uint64_t k = okey(v, pess);
    if (ok && k < kstar) {
      lt += g;
      vgl = fma(g, v, vgl);
    }
    if (ok && k == kstar && i < pos) pos = i;
  });
  lt = wsum(lt);
  vgl = wsum(vgl);
  pos = (int)wmin((uint64_t)(unsigned)pos);
  if (lane == 0) d.tpos[j] = pos;
  return base + vgl + (rem - lt) * ovalue(kstar, pess);
}

template <int R>
__device__ __forceinline__ double col_value_reg(const Dev& d, int j, int a, int m, const double* V, bool pess) {
  const int lane = threadIdx.x & 63;
  RegCol<R> col;
  col.m = m;
  double base = 0.0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int i = lane + 64 * r;
    if (i < m) {
      const double v = V[d.rowval[a + i]];
      col.v[r] = v;
      col.g[r] = d.gap[a + i];
      base = fma(d.lower[a + i], v, base);
    } else {
      col.v[r] = 0.0;
      col.g[r] = 0.0;
    }
  }
  base = wsum(base);
  return col_finish(d, j, a, col, V, base, pess);
}

__device__ __forceinline__ double col_value_stream(const Dev& d, int j, int a, int m, const double* V, bool pess) {
  StreamCol col{d.rowval + a, d.gap + a, V, m};
  const int lane = threadIdx.x & 63;
  double base = 0.0;
  for (int c = 0; c < m; c += 64) {
    const int i = c + lane;
    if (i < m) base = fma(d.lower[a + i], V[d.rowval[a + i]], base);
  }
  base = wsum(base);
  return col_finish(d, j, a, col, V, base, pess);
}

// Column classes by length: up to 64 R destinations stay in registers
// (R = 1, 2, 3, 4, 6, 8, 12, 16: steps of at most half the length, so that a
// column's registers are not far above what it needs); longer columns are
// re-read on every pass.  A kernel instance handles the states whose longest
// column is in class RMAX, so that its register budget (and occupancy) is set
// by that class only.
constexpr int kNumClasses = 9;
constexpr int kClassR[kNumClasses] = {1, 2, 3, 4, 6, 8, 12, 16, 0};
__host__ __device__ constexpr int class_rmax(int c) { return kClassR[c]; }
__host__ __device__ inline int class_of_len(int m) {
  return m <= 64 ? 0 : m <= 128 ? 1 : m <= 192 ? 2 : m <= 256 ? 3 : m <= 384 ? 4 : m <= 512 ? 5 : m <= 768 ? 6
         : m <= 1024 ? 7 : 8;
}

template <int RMAX>
__device__ __forceinline__ double col_value(const Dev& d, int j, const double* V, bool pess) {
  const int a = d.colptr[j];
  const int m = d.colptr[j + 1] - a;
  if (m <= 0) return 0.0;
  if (m <= 64) return col_value_reg<1>(d, j, a, m, V, pess);
  if (RMAX >= 2 && m <= 128) return col_value_reg<(RMAX >= 2 ? 2 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 3 && m <= 192) return col_value_reg<(RMAX >= 3 ? 3 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 4 && m <= 256) return col_value_reg<(RMAX >= 4 ? 4 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 6 && m <= 384) return col_value_reg<(RMAX >= 6 ? 6 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 8 && m <= 512) return col_value_reg<(RMAX >= 8 ? 8 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 12 && m <= 768) return col_value_reg<(RMAX >= 12 ? 12 : 1)>(d, j, a, m, V, pess);
  if (RMAX >= 16 && m <= 1024) return col_value_reg<(RMAX >= 16 ? 16 : 1)>(d, j, a, m, V, pess);
  return col_value_stream(d, j, a, m, V, pess);
}

// Occupancy floors per class (waves per SIMD): the loads of a column are
// in flight while the wave waits, so waves are what hides HBM latency.  The
// floors are measured: R = 6 gains from 7 waves despite a few spilled values
// (0.246 against 0.249 ms per iteration at 376 destinations per column),
// while R = 8 and R = 12 lose with spills (0.150 against 0.162 ms at 451, and
// 0.214 against 0.249 ms at 701, at 6 and 5 waves instead of 5 and 4).
constexpr int step_waves(int rmax) {
  return rmax <= 3 ? 8 : rmax == 4 ? 7 : rmax == 6 ? 7 : rmax == 8 ? 5 : rmax == 12 ? 4 : 3;
}

// One iteration of Eq. 2: one wavefront per state.
template <int RMAX>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(step_waves(RMAX)))) void vi_step_kernel(
    const StepArgs A) {
  __shared__ double wres[kWavesPerBlock];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int ws = blockIdx.x * kWavesPerBlock + w;
  double delta = 0.0;
  if (ws < A.n_list) {  // wave-uniform
    const int s = A.states[ws];
    const double fx = A.fixed ? A.fixed[s] : NAN;
    double nv;
    int arg = 0;
    if (!isnan(fx)) {
      nv = fx;
    } else {
      const int c0 = A.d.stateptr[s], c1 = A.d.stateptr[s + 1];
      double best = 0.0;
      for (int j = c0; j < c1; ++j) {
        const double q = col_value<RMAX>(A.d, j, A.Vin, A.pessimistic != 0);
        if (j == c0 || (A.maximize ? q > best : q < best)) {
          best = q;
          arg = j - c0;
        }
      }
      nv = A.reward ? A.reward[s] + A.discount * best : best;
    }
    if (lane == 0) {
      A.Vout[s] = nv;
      if (A.policy) A.policy[(size_t)s * A.policy_stride] = arg;
    }
    delta = fabs(nv - A.Vin[s]);
  }
  if (A.partial) {
    if (lane == 0) wres[w] = delta;
    __syncthreads();
    if (threadIdx.x == 0) {
      double mx = wres[0];
      for (int i = 1; i < kWavesPerBlock; ++i) mx = fmax(mx, wres[i]);
      A.partial[blockIdx.x] = mx;
    }
  }
}

// Maximum of the per-block residuals (one block).
__global__ __launch_bounds__(256) void max_kernel(const double* partial, int n, double* out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) mx = fmax(mx, partial[i]);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace
}  // namespace imdp

using namespace imdp;

struct imdp_vi {
  int device = 0;
  int n_states = 0, n_columns = 0;
  int64_t nnz = 0;
  hipStream_t stream = nullptr;
  int *stateptr = nullptr, *colptr = nullptr, *rowval = nullptr, *tpos = nullptr;
  double *lower = nullptr, *gap = nullptr, *rem = nullptr, *gtot = nullptr;
  double *V0 = nullptr, *V1 = nullptr, *fixed = nullptr, *reward = nullptr, *partial = nullptr, *res = nullptr;
  int* policy = nullptr;
  size_t policy_cap = 0;
  int* slist = nullptr;                // states grouped by column class
  int class_off[kNumClasses + 1] = {}; // class c: slist[class_off[c] .. class_off[c+1])
  int total_blocks = 0;
  double* host_res = nullptr;  // pinned
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

struct DevGuard {
  int prev = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void release(imdp_vi* h) {
  for (void* p : {(void*)h->slist, (void*)h->stateptr, (void*)h->colptr, (void*)h->rowval, (void*)h->tpos, (void*)h->lower,
                  (void*)h->gap, (void*)h->rem, (void*)h->gtot, (void*)h->V0, (void*)h->V1, (void*)h->fixed,
                  (void*)h->reward, (void*)h->partial, (void*)h->res, (void*)h->policy})
    if (p) (void)hipFree(p);
  if (h->host_res) (void)hipHostFree(h->host_res);
  if (h->ev0) (void)hipEventDestroy(h->ev0);
  if (h->ev1) (void)hipEventDestroy(h->ev1);
  if (h->stream) (void)hipStreamDestroy(h->stream);
}

template <typename T>
bool dev_alloc(T** p, size_t n) {
  return hipMalloc((void**)p, sizeof(T) * (n ? n : 1)) == hipSuccess;
}

int blocks_of(int n_states) { return (n_states + kWavesPerBlock - 1) / kWavesPerBlock; }

using StepFn = void (*)(const StepArgs);
const StepFn kStep[kNumClasses] = {vi_step_kernel<1>, vi_step_kernel<2>,  vi_step_kernel<3>,
                                   vi_step_kernel<4>, vi_step_kernel<6>,  vi_step_kernel<8>,
                                   vi_step_kernel<12>, vi_step_kernel<16>, vi_step_kernel<0>};

}  // namespace

extern "C" int imdp_vi_create(int32_t device, const imdp_model* M, imdp_vi** out) {
  if (!M || !out) return IMDP_EINVAL;
  *out = nullptr;
  const int S = M->n_states, C = M->n_columns;
  const int64_t nnz = M->nnz;
  if (S <= 0 || C < 0 || nnz < 0 || !M->stateptr || !M->colptr) return IMDP_EINVAL;
  if (nnz > 0 && (!M->rowval || !M->lower || !M->upper)) return IMDP_EINVAL;
  if (nnz > (int64_t)INT32_MAX || (int64_t)S * kWavesPerBlock > (int64_t)INT32_MAX) return IMDP_EUNSUPPORTED;
  if (M->stateptr[0] != 0 || M->stateptr[S] != C || M->colptr[0] != 0 || M->colptr[C] != nnz) return IMDP_EINVAL;
  for (int s = 0; s < S; ++s)
    if (M->stateptr[s + 1] < M->stateptr[s]) return IMDP_EINVAL;
  for (int j = 0; j < C; ++j)
    if (M->colptr[j + 1] < M->colptr[j]) return IMDP_EINVAL;
  std::vector<double> gap((size_t)nnz), rem((size_t)C), gtot((size_t)C);
  // states by the class of their longest column
  std::vector<int> cls((size_t)S);
  int cnt[kNumClasses] = {};
  for (int s = 0; s < S; ++s) {
    int mx = 0;
    for (int j = M->stateptr[s]; j < M->stateptr[s + 1]; ++j) mx = std::max(mx, M->colptr[j + 1] - M->colptr[j]);
    cls[s] = class_of_len(mx);
    cnt[cls[s]]++;
  }
  for (int j = 0; j < C; ++j) {
    double sl = 0.0, sg = 0.0;
    for (int64_t e = M->colptr[j]; e < M->colptr[j + 1]; ++e) {
      const double lo = M->lower[e], up = M->upper[e];
      if (!(lo >= 0.0) || !(up <= 1.0) || !(lo <= up) || M->rowval[e] < 0 || M->rowval[e] >= S) return IMDP_EINVAL;
      gap[e] = up - lo;
      sl += lo;
      sg += gap[e];
    }
    rem[j] = 1.0 - sl;
    gtot[j] = sg;
  }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IMDP_EINVAL;
  DevGuard dg(device);
  imdp_vi* h = new (std::nothrow) imdp_vi();
  if (!h) return IMDP_ENOMEM;
  h->device = device;
  h->n_states = S;
  h->n_columns = C;
  h->nnz = nnz;
  std::vector<int> slist((size_t)S);
  {
    int pos[kNumClasses];
    h->class_off[0] = 0;
    for (int c = 0; c < kNumClasses; ++c) {
      h->class_off[c + 1] = h->class_off[c] + cnt[c];
      pos[c] = h->class_off[c];
      h->total_blocks += blocks_of(cnt[c]);
    }
    for (int s = 0; s < S; ++s) slist[pos[cls[s]]++] = s;
  }
  const int nb = h->total_blocks;
  bool ok = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking) == hipSuccess;
  ok = ok && dev_alloc(&h->stateptr, S + 1) && dev_alloc(&h->colptr, (size_t)C + 1) &&
       dev_alloc(&h->rowval, (size_t)nnz) && dev_alloc(&h->lower, (size_t)nnz) && dev_alloc(&h->gap, (size_t)nnz) &&
       dev_alloc(&h->rem, (size_t)C) && dev_alloc(&h->gtot, (size_t)C) && dev_alloc(&h->tpos, (size_t)C) &&
       dev_alloc(&h->V0, S) && dev_alloc(&h->V1, S) && dev_alloc(&h->fixed, S) && dev_alloc(&h->reward, S) &&
       dev_alloc(&h->partial, nb) && dev_alloc(&h->res, 1) && dev_alloc(&h->slist, S);
  ok = ok && hipHostMalloc((void**)&h->host_res, sizeof(double), hipHostMallocDefault) == hipSuccess;
  ok = ok && hipEventCreate(&h->ev0) == hipSuccess && hipEventCreate(&h->ev1) == hipSuccess;
  if (!ok) {
    release(h);
    delete h;
    return IMDP_ENOMEM;
  }
  hipError_t e = hipMemcpy(h->stateptr, M->stateptr, sizeof(int) * (S + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->colptr, M->colptr, sizeof(int) * ((size_t)C + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(h->rowval, M->rowval, sizeof(int) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(h->lower, M->lower, sizeof(double) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess && nnz) e = hipMemcpy(h->gap, gap.data(), sizeof(double) * nnz, hipMemcpyHostToDevice);
  if (e == hipSuccess && C) e = hipMemcpy(h->rem, rem.data(), sizeof(double) * C, hipMemcpyHostToDevice);
  if (e == hipSuccess && C) e = hipMemcpy(h->gtot, gtot.data(), sizeof(double) * C, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->slist, slist.data(), sizeof(int) * S, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    release(h);
    delete h;
    return IMDP_EDEVICE;
  }
  *out = h;
  return IMDP_OK;
}

extern "C" int imdp_vi_run(imdp_vi* h, const imdp_spec* sp, double* V_out, int32_t* policy_out, imdp_result* out) {
  if (!h || !sp || !V_out) return IMDP_EINVAL;
  const int S = h->n_states;
  if (sp->property != IMDP_REACH && sp->property != IMDP_REACH_AVOID && sp->property != IMDP_REWARD)
    return IMDP_EINVAL;
  if (sp->horizon < 0 || (sp->horizon == 0 && !(sp->eps > 0.0))) return IMDP_EINVAL;
  const bool reward = sp->property == IMDP_REWARD;
  if (reward && (!sp->reward || !(sp->discount >= 0.0) || !(sp->discount <= 1.0))) return IMDP_EINVAL;
  if (sp->n_targets < 0 || (sp->n_targets > 0 && !sp->targets)) return IMDP_EINVAL;
  if (sp->property == IMDP_REACH_AVOID && (sp->n_avoid < 0 || (sp->n_avoid > 0 && !sp->avoid))) return IMDP_EINVAL;
  // V_0 and the states the recursion does not update
  std::vector<double> v0((size_t)S, 0.0), fixed((size_t)S, NAN);
  if (reward) {
    for (int s = 0; s < S; ++s) {
      if (!std::isfinite(sp->reward[s])) return IMDP_EINVAL;
      v0[s] = sp->reward[s];
    }
  } else {
    if (sp->property == IMDP_REACH_AVOID)
      for (int i = 0; i < sp->n_avoid; ++i) {
        const int s = sp->avoid[i];
        if (s < 0 || s >= S) return IMDP_EINVAL;
        fixed[s] = 0.0;
      }
    for (int i = 0; i < sp->n_targets; ++i) {
      const int s = sp->targets[i];
      if (s < 0 || s >= S) return IMDP_EINVAL;
      fixed[s] = 1.0;
    }
    for (int s = 0; s < S; ++s)
      if (!std::isnan(fixed[s])) v0[s] = fixed[s];
  }
  const int K = sp->horizon;
  const int maxit = K > 0 ? K : (sp->max_iterations > 0 ? sp->max_iterations : 100000);
  DevGuard dg(h->device);
  hipStream_t st = h->stream;
  hipError_t e = hipMemcpyAsync(h->V0, v0.data(), sizeof(double) * S, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->fixed, fixed.data(), sizeof(double) * S, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && reward)
    e = hipMemcpyAsync(h->reward, sp->reward, sizeof(double) * S, hipMemcpyHostToDevice, st);
  if (e == hipSuccess && h->n_columns) e = hipMemsetAsync(h->tpos, 0, sizeof(int) * h->n_columns, st);
  const size_t pol_n = policy_out ? (K > 0 ? (size_t)S * K : (size_t)S) : 0;
  if (e == hipSuccess && pol_n > h->policy_cap) {
    if (h->policy) (void)hipFree(h->policy);
    h->policy = nullptr;
    h->policy_cap = 0;
    if (hipMalloc((void**)&h->policy, sizeof(int) * pol_n) != hipSuccess) return IMDP_ENOMEM;
    h->policy_cap = pol_n;
  }
  // the host's V_0 buffer must stay valid until the copy ran
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return IMDP_EDEVICE;

  StepArgs A{};
  A.d = Dev{h->stateptr, h->colptr, h->rowval, h->lower, h->gap, h->rem, h->gtot, h->tpos};
  A.fixed = reward ? nullptr : h->fixed;
  A.reward = reward ? h->reward : nullptr;
  A.discount = sp->discount;
  A.pessimistic = sp->pessimistic ? 1 : 0;
  A.maximize = sp->maximize ? 1 : 0;
  const int nb = h->total_blocks;
  double* cur = h->V0;
  double* nxt = h->V1;
  int it = 0;
  double residual = 0.0;
  e = hipEventRecord(h->ev0, st);
  while (e == hipSuccess && it < maxit) {
    ++it;
    A.Vin = cur;
    A.Vout = nxt;
    if (policy_out && K > 0) {
      A.policy = h->policy + (K - it);  // time t = K - it
      A.policy_stride = K;
    } else if (policy_out) {
      A.policy = h->policy;
      A.policy_stride = 1;
    } else {
      A.policy = nullptr;
    }
    const bool check = K == 0 || it == K;
    int boff = 0;
    for (int c = 0; c < kNumClasses && e == hipSuccess; ++c) {
      const int n = h->class_off[c + 1] - h->class_off[c];
      if (n == 0) continue;
      A.states = h->slist + h->class_off[c];
      A.n_list = n;
      A.partial = check ? h->partial + boff : nullptr;
      hipLaunchKernelGGL(kStep[c], dim3(blocks_of(n)), dim3(kThreads), 0, st, A);
      e = hipGetLastError();
      boff += blocks_of(n);
    }
    if (e == hipSuccess && check) {
      hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, h->partial, nb, h->res);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(h->host_res, h->res, sizeof(double), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e == hipSuccess) residual = *h->host_res;
    }
    double* t = cur;
    cur = nxt;
    nxt = t;
    if (K == 0 && residual < sp->eps) break;
  }
  if (e == hipSuccess) e = hipEventRecord(h->ev1, st);
  if (e == hipSuccess) e = hipMemcpyAsync(V_out, cur, sizeof(double) * S, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && policy_out)
    e = hipMemcpyAsync(policy_out, h->policy, sizeof(int) * pol_n, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return IMDP_EDEVICE;
  if (out) {
    out->iterations = it;
    out->residual = residual;
    float ms = 0.0f;
    out->kernel_ms = hipEventElapsedTime(&ms, h->ev0, h->ev1) == hipSuccess ? (double)ms : -1.0;
  }
  return IMDP_OK;
}

extern "C" int imdp_vi_destroy(imdp_vi* h) {
  if (!h) return IMDP_EINVAL;
  {
    DevGuard dg(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    release(h);
  }
  delete h;
  return IMDP_OK;
}
