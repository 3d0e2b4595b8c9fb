// Blocked Householder reduction to upper Hessenberg form for large models
// (n > 256), spread over the whole GPU as a sequence of kernels on one stream.
//
// The reflectors are those of the unblocked reduction (Golub & Van Loan,
// Matrix Computations, 4th ed., Algorithm 7.4.2; LAPACK dlarfg sign
// convention), grouped into panels of nb = 32 columns.  The panel's
// reflectors are accumulated in compact WY form Q = I - V T V^T (T upper
// triangular) together with Y = M V T (Golub & Van Loan sec. 5.1.7; the
// panel scheme of Quintana-Orti and van de Geijn for the Hessenberg case),
// so that the trailing matrix is touched only once per panel:
//
//   panel column c = k + j:
//     b   = M(:, c) - Y V(c, :)^T                 (earlier right updates)
//     b   = b - V T^T V^T b                       (earlier left updates)
//     v_j, tau_j from b (rows c+1 ..);  w = V^T v_j
//     Y(:, j) = tau_j (M v_j - Y w),  T(:, j) = [-tau_j T w ; tau_j]
//   end of panel:
//     M(:, trailing) -= Y V(trailing, :)^T        (right, all n+p rows)
//     M(rows k+1 .., trailing) -= V T^T V^T M(..)  (left, with the B columns)
//
// M is the augmented (n+p) x (n+m) matrix [[A, B], [C, *]] (column-major in
// the job's scratch area), so Q^T B and C Q come out of the same updates.
//
// Kernels, per panel column: blk_panel (one workgroup: the left update of
// column c from the per-block partial products V^T b, the reflector, w and
// T) and blk_rows (16-row blocks: the product of the panel-start matrix with
// v_j, the bandwidth-heavy part; it finishes Y(:, j) for its rows, forms the
// next panel column's b = M(:, c+1) - Y V(c+1, :)^T there and its partial
// V^T b, so that every row-parallel step runs on the whole GPU and each sum
// has a fixed order).  Per panel: blk_right and blk_left, the rank-nb updates
// of the trailing matrix, on the float64 matrix cores (v_mfma_f64_16x16x4f64).
#include <algorithm>

#include "dpp.h"
#include "lti_kernels.h"

namespace lti {

namespace {

constexpr int kNB = 32;          // panel width
constexpr int kPThreads = 1024;  // blk_panel: one workgroup
constexpr int kRowBlock = 64;    // rows per workgroup (blk_right); row padding
constexpr int kRows = 16;        // rows per workgroup (blk_rows)
constexpr int kLeftCols = 16;    // columns per workgroup (blk_left)

struct BlkLayout {
  int ldm, ldv;  // leading dimensions of M, Y, b (rows) and V
  int nrb;       // row blocks of blk_rows
  size_t M, V, Y, T, tau, w, b, upart, total;  // offsets in doubles
};

__host__ __device__ inline BlkLayout blk_layout(int n, int m, int p) {
  BlkLayout L;
  L.ldm = ((n + p) + kRowBlock - 1) / kRowBlock * kRowBlock;
  L.ldv = (n + 15) & ~15;
  size_t o = 0;
  L.M = o;
  o += (size_t)L.ldm * (n + m);
  L.V = o;
  o += (size_t)L.ldv * kNB;
  L.Y = o;
  o += (size_t)L.ldm * kNB;
  L.T = o;
  o += kNB * kNB;
  L.tau = o;
  o += kNB;
  L.w = o;
  o += kNB;
  L.b = o;  // the next panel column, updated by earlier right updates
  o += (size_t)L.ldm;
  L.nrb = L.ldm / kRows;
  L.upart = o;  // per row block: V^T b over its rows
  o += (size_t)L.nrb * kNB;
  L.total = o;
  return L;
}

// Up to kBlkBatch models per launch, model z on blockIdx.z: the per-column
// kernels are latency chains that use a few CUs, so the models of one
// admission pass run them side by side.  Models of different sizes share the
// column loop of the largest; a model's kernels return once its own panel
// (or column) range is done.
constexpr int kBlkBatch = 8;
struct BlkArgs {
  ReduceJob job[kBlkBatch];
  int k;  // first column of the panel
  int j;  // column within the panel
};
static_assert(sizeof(BlkArgs) <= 3072, "blocked reduction arguments must stay small");

// Width of the panel starting at column k of an n-state model (<= 0 once
// its last reflector, column n-3, is done).
__host__ __device__ inline int blk_nbk(int n, int k) { return (kNB < n - 2 - k) ? kNB : n - 2 - k; }

struct Blk {
  int n, m, p, N, C;
  BlkLayout L;
  double *M, *V, *Y, *T, *tau, *w, *b, *upart;
  __device__ explicit Blk(const ReduceJob& job) {
    n = job.out.n;
    m = job.out.m;
    p = job.out.p;
    N = n + p;
    C = n + m;
    L = blk_layout(n, m, p);
    double* W = job.work;
    M = W + L.M;
    V = W + L.V;
    Y = W + L.Y;
    T = W + L.T;
    tau = W + L.tau;
    w = W + L.w;
    b = W + L.b;
    upart = W + L.upart;
  }
};

// M = [[A, B], [C, 0]], padding rows zero.
// The solved system is also kept as given (A0, B0, C0) for the extended
// refinement.
__global__ __launch_bounds__(256) void blk_load(const BlkArgs a) {
  const ReduceJob& job = a.job[blockIdx.z];
  const Blk b(job);
  const ModelIn in(job);
  const ReducedModel& o = job.out;
  const size_t total = (size_t)b.L.ldm * b.C;
  for (size_t idx = (size_t)blockIdx.x * 256 + threadIdx.x; idx < total; idx += (size_t)gridDim.x * 256) {
    const int i = (int)(idx % b.L.ldm);
    const int c = (int)(idx / b.L.ldm);
    double x = 0.0;
    if (i < b.n) {
      if (c < b.n) {
        x = in.a(i, c);
        o.A0[(size_t)c * b.n + i] = x;
      } else {
        x = in.b(i, c - b.n);
        o.B0[(size_t)(c - b.n) * b.n + i] = x;
      }
    } else if (i < b.N && c < b.n) {
      x = in.c(i - b.n, c);
      o.C0[(size_t)(i - b.n) * b.n + c] = x;
    }
    b.M[idx] = x;
  }
}

// Column j of the panel.  On entry B.b holds b = M(:, c) - Y V(c, :)^T (for
// j = 0: M(:, c) itself) and, for j > 0, B.upart the per-row-block partial
// sums of V^T b over rows k+1 .. n-1.
__global__ __launch_bounds__(kPThreads) void blk_panel(const BlkArgs a) {
  __shared__ double bv[kMaxReduceN + kRowBlock];  // the working column b
  __shared__ double red[kNB];                      // u, then w
  __shared__ double zz[kNB];                       // T^T u
  __shared__ double sc[4];                         // beta, tau, scale
  const ReduceJob& job = a.job[blockIdx.z];
  const Blk B(job);
  const int n = B.n, N = B.N, ldv = B.L.ldv, ldm = B.L.ldm;
  const int k = a.k, j = a.j, c = k + j;
  if (j >= blk_nbk(n, k)) return;  // this model's columns are done (uniform)
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  constexpr int kWavesP = kPThreads / 64;

  for (int i = tid; i < N; i += kPThreads) bv[i] = (j == 0) ? B.M[(size_t)c * ldm + i] : B.b[i];
  if (j > 0) {
    {  // u = V^T b from the row blocks' partial sums: 32 threads per
       // reflector (one half wavefront), each a fixed stride of blocks, then
       // a fixed-order DPP sum over the 32
      const int l = tid >> 5, t32 = tid & 31;
      double u = 0.0;
      if (l < j)
        for (int rb = t32; rb < B.L.nrb; rb += 32) u += B.upart[(size_t)rb * kNB + l];
      u = group_sum_dpp<16>(u);
      u += dpp<kDppRowBcast15, 0xa>(u);  // rows 1, 3 add rows 0, 2
      if (l < j && t32 == 31) red[l] = u;
    }
    __syncthreads();
    if (tid < j) {  // z = T^T u
      double z = 0.0;
#pragma unroll
      for (int l2 = 0; l2 < kNB; ++l2)
        if (l2 <= tid) z = fma(B.T[l2 + tid * kNB], red[l2], z);
      zz[tid] = z;
    }
    __syncthreads();
    for (int i = k + 1 + tid; i < n; i += kPThreads) {
      double x = bv[i];
#pragma unroll
      for (int l = 0; l < kNB; ++l)
        if (l < j) x = fma(-B.V[(size_t)l * ldv + i], zz[l], x);
      bv[i] = x;
    }
  }
  __syncthreads();
  // reflector of b(c+1 .. n-1)
  if (wv == 0) {
    double ss = 0.0;
    for (int i = c + 2 + lane; i < n; i += 64) ss = fma(bv[i], bv[i], ss);
    ss = wave_sum_dpp(ss);
    if (lane == 0) {
      const double alpha = bv[c + 1];
      double beta = alpha, tau = 0.0, scale = 0.0;
      if (ss != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, ss));
        beta = (alpha >= 0.0) ? -nrm : nrm;
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      sc[0] = beta;
      sc[1] = tau;
      sc[2] = scale;
    }
  }
  __syncthreads();
  const double beta = sc[0], tau = sc[1], scale = sc[2];
  // column c is final: rows up to c, beta below the diagonal, zeros, C rows
  for (int i = tid; i < N; i += kPThreads) {
    double x;
    if (i <= c)
      x = bv[i];
    else if (i == c + 1)
      x = beta;
    else if (i < n)
      x = 0.0;
    else
      x = bv[i];
    B.M[(size_t)c * ldm + i] = x;
  }
  // the panel's V, and every reflector kept in the reduced model
  const int64_t vo = voff(n, c) - (c + 2);
  for (int i = k + 1 + tid; i < n; i += kPThreads) {
    const double vi = (i <= c) ? 0.0 : (i == c + 1) ? 1.0 : bv[i] * scale;
    B.V[(size_t)j * ldv + i] = vi;
    if (i >= c + 2) job.out.V[vo + i] = vi;
  }
  if (tid == 0) {
    B.tau[j] = tau;
    job.out.tau[c] = tau;
  }
  __syncthreads();
  if (j > 0) {
    // w = V^T v_j over rows c+1 .. n-1
    for (int l = wv; l < j; l += kWavesP) {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int i = c + 1 + lane;
      for (; i + 3 * 64 < n; i += 4 * 64)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          s4[q] = fma(B.V[(size_t)l * ldv + i + 64 * q], B.V[(size_t)j * ldv + i + 64 * q], s4[q]);
      for (; i < n; i += 64) s4[0] = fma(B.V[(size_t)l * ldv + i], B.V[(size_t)j * ldv + i], s4[0]);
      const double s = wave_sum_dpp((s4[0] + s4[1]) + (s4[2] + s4[3]));
      if (lane == 0) red[l] = s;
    }
    __syncthreads();
    if (tid < j) {  // T(0:j, j) = -tau T w; w kept for Y(:, j)
      double t = 0.0;
#pragma unroll
      for (int l2 = 0; l2 < kNB; ++l2)
        if (l2 >= tid && l2 < j) t = fma(B.T[tid + l2 * kNB], red[l2], t);
      B.T[tid + j * kNB] = -tau * t;
      B.w[tid] = red[tid];
    }
  }
  if (tid == 0) B.T[j + j * kNB] = tau;
}

// Rows i of one 16-row block (256 threads: 16 rows x 16 column lanes):
//   Y(i, j) = tau_j (sum_{col > c} M(i, col) v_j(col) - Y(i, 0:j) w)
// and, unless j is the panel's last column,
//   b(i) = M(i, c+1) - Y(i, 0:j+1) V(c+1, 0:j+1)^T
//   upart(block, l) = sum over the block's rows in k+1 .. n-1 of V(i, l) b(i).
__global__ __launch_bounds__(256) void blk_rows(const BlkArgs a) {
  __shared__ double red[16][kRows + 1];
  __shared__ double sb[kRows];
  const Blk B(a.job[blockIdx.z]);
  const int n = B.n, ldm = B.L.ldm, ldv = B.L.ldv;
  const int k = a.k, j = a.j, c = k + j;
  const int nbk = blk_nbk(n, k);
  if (j >= nbk || (int)blockIdx.x >= B.L.nrb) return;  // uniform
  const int tid = threadIdx.x, r = tid & (kRows - 1), cl = tid >> 4;  // row, column lane
  const int i = blockIdx.x * kRows + r;  // < ldm
  const double* vj = B.V + (size_t)j * ldv;
  // sixteen independent partial sums keep sixteen loads in flight per lane
  double s16[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) s16[q] = 0.0;
  int col = c + 1 + cl;
  for (; col + 15 * 16 < n; col += 16 * 16)
#pragma unroll
    for (int q = 0; q < 16; ++q) s16[q] = fma(B.M[(size_t)(col + 16 * q) * ldm + i], vj[col + 16 * q], s16[q]);
#pragma unroll
  for (int q = 0; q < 16; ++q) {  // the remainder, still all loads at once
    const int cq = col + 16 * q;
    if (cq < n) s16[q] = fma(B.M[(size_t)cq * ldm + i], vj[cq], s16[q]);
  }
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1)
#pragma unroll
    for (int q = 0; q < h; ++q) s16[q] += s16[q + h];
  red[cl][r] = s16[0];
  __syncthreads();
  if (cl == 0) {
    // this row of Y (issued together: the loop bound is the panel width)
    double yr[kNB];
#pragma unroll
    for (int l = 0; l < kNB; ++l) yr[l] = (l < j) ? B.Y[(size_t)l * ldm + i] : 0.0;
    double y = 0.0;
#pragma unroll
    for (int q = 0; q < 16; ++q) y += red[q][r];
#pragma unroll
    for (int l = 0; l < kNB; ++l)
      if (l < j) y = fma(-yr[l], B.w[l], y);
    y *= B.tau[j];
    B.Y[(size_t)j * ldm + i] = y;
    if (j + 1 < nbk) {
      const int c1 = c + 1;
      double x = B.M[(size_t)c1 * ldm + i];
#pragma unroll
      for (int l = 0; l < kNB; ++l)
        if (l < j) x = fma(-yr[l], B.V[(size_t)l * ldv + c1], x);
      x = fma(-y, vj[c1], x);
      B.b[i] = x;
      sb[r] = (i > k && i < n) ? x : 0.0;
    }
  }
  if (j + 1 >= nbk) return;  // uniform
  __syncthreads();
  // partial V^T b for l = 0 .. j over this block's rows
  for (int l = tid; l <= j; l += 256) {
    double u = 0.0;
    const int i0 = blockIdx.x * kRows;
#pragma unroll
    for (int q = 0; q < kRows; ++q) {
      const int ii = i0 + q;
      if (ii > k && ii < n) u = fma(B.V[(size_t)l * ldv + ii], sb[q], u);
    }
    B.upart[(size_t)blockIdx.x * kNB + l] = u;
  }
}

// M(:, k+nbk .. n-1) -= Y V(k+nbk .. n-1, :)^T on the float64 matrix cores.
// A 64 x 64 tile per workgroup; wavefront w owns rows 16 w .. 16 w + 15 and
// the tile's four 16 x 16 column blocks.  v_mfma_f64_16x16x4f64 (lane l,
// checked on the device): A operand = A(l % 16, l / 16), B operand =
// B(l / 16, l % 16), result element q = D((l / 16) + 4 q, l % 16).
typedef double dbl4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void blk_right(const BlkArgs a) {
  __shared__ double sY[kNB][kRowBlock + 1];
  __shared__ double sV[kNB][kRowBlock + 1];
  const Blk B(a.job[blockIdx.z]);
  const int n = B.n, ldm = B.L.ldm, ldv = B.L.ldv;
  const int nbk = blk_nbk(n, a.k), cstart = a.k + nbk;
  const int r0 = blockIdx.x * kRowBlock, cc0 = cstart + blockIdx.y * 64;
  if (nbk <= 0 || r0 >= ldm || cc0 >= n) return;  // uniform
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kNB * kRowBlock; idx += 256) {
    const int l = idx / kRowBlock, r = idx % kRowBlock;
    sY[l][r] = (l < nbk) ? B.Y[(size_t)l * ldm + r0 + r] : 0.0;
    const int col = cc0 + r;
    sV[l][r] = (l < nbk && col < n) ? B.V[(size_t)l * ldv + col] : 0.0;
  }
  __syncthreads();
  const int lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) acc[cb] = dbl4{0.0, 0.0, 0.0, 0.0};
  for (int kk = 0; kk < nbk; kk += 4) {  // rows of sY/sV past nbk are zero
    const double av = sY[kk + lk][16 * wv + lr];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const double bv = sV[kk + lk][16 * cb + lr];
      acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[cb], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int col = cc0 + 16 * cb + lr;
    if (col >= n) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = r0 + 16 * wv + lk + 4 * q;
      if (i < B.N) B.M[(size_t)col * ldm + i] -= acc[cb][q];
    }
  }
}

// M(k+1 .. n-1, cols) -= V T^T V^T M(k+1 .. n-1, cols) for kLeftCols = 16
// trailing columns (B's included) per workgroup, both products on the
// float64 matrix cores (layout as in blk_right):
//   W = V^T M: 64-row blocks staged in LDS, each wavefront takes four of the
//     block's sixteen 4-row steps, two 16-row halves of W (reflectors 0-15,
//     16-31) per wavefront, partial W summed over the wavefronts in LDS;
//   Z = T^T W on the vector unit;  M -= V Z: 16-row blocks, one wavefront
//     each, the A operand read straight from V.
__global__ __launch_bounds__(256) void blk_left(const BlkArgs a) {
  __shared__ double sV[kRowBlock][kNB + 1];
  __shared__ double sM[kRowBlock][kLeftCols + 1];
  __shared__ double sW[4][kNB][kLeftCols + 1];
  const Blk B(a.job[blockIdx.z]);
  const int n = B.n, C = B.C, ldm = B.L.ldm, ldv = B.L.ldv;
  const int k = a.k, nbk = blk_nbk(n, k);
  const int col0 = k + nbk + blockIdx.x * kLeftCols;
  if (nbk <= 0 || col0 >= C) return;  // uniform
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;
  dbl4 acc[2] = {dbl4{0.0, 0.0, 0.0, 0.0}, dbl4{0.0, 0.0, 0.0, 0.0}};
  for (int rb = k + 1; rb < n; rb += kRowBlock) {
    for (int idx = tid; idx < kRowBlock * kNB; idx += 256) {
      const int r = idx % kRowBlock, ll = idx / kRowBlock;
      const int i = rb + r;
      sV[r][ll] = (i < n && ll < nbk) ? B.V[(size_t)ll * ldv + i] : 0.0;
    }
    for (int idx = tid; idx < kRowBlock * kLeftCols; idx += 256) {
      const int r = idx % kRowBlock, qq = idx / kRowBlock;
      const int i = rb + r, col = col0 + qq;
      sM[r][qq] = (i < n && col < C) ? B.M[(size_t)col * ldm + i] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int r = 16 * wv + 4 * st + lk;  // this lane's row of the K step
      const double bm = sM[r][lr];
#pragma unroll
      for (int lb = 0; lb < 2; ++lb)
        acc[lb] = __builtin_amdgcn_mfma_f64_16x16x4f64(sV[r][16 * lb + lr], bm, acc[lb], 0, 0, 0);
    }
    __syncthreads();
  }
  // acc[lb][q] = partial W(16 lb + lk + 4 q, lr)
#pragma unroll
  for (int lb = 0; lb < 2; ++lb)
#pragma unroll
    for (int q = 0; q < 4; ++q) sW[wv][16 * lb + lk + 4 * q][lr] = acc[lb][q];
  __syncthreads();
  // Z = T^T W, written over sW[0]
  double z[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + 256 * h, l = e >> 4, qq = e & 15;  // 512 entries of Z
    double zv = 0.0;
    if (l < nbk)
      for (int l2 = 0; l2 <= l; ++l2) {
        const double wsum = (sW[0][l2][qq] + sW[1][l2][qq]) + (sW[2][l2][qq] + sW[3][l2][qq]);
        zv = fma(B.T[l2 + l * kNB], wsum, zv);
      }
    z[h] = zv;
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int e = tid + 256 * h;
    sW[0][e >> 4][e & 15] = z[h];
  }
  __syncthreads();
  // M -= V Z, one 16-row block per wavefront at a time
  for (int i0 = k + 1 + 16 * wv; i0 < n; i0 += 64) {
    dbl4 d = {0.0, 0.0, 0.0, 0.0};
    for (int kk = 0; kk < nbk; kk += 4) {
      const int i = i0 + lr, ll = kk + lk;
      const double av = (i < n && ll < nbk) ? B.V[(size_t)ll * ldv + i] : 0.0;
      d = __builtin_amdgcn_mfma_f64_16x16x4f64(av, sW[0][ll][lr], d, 0, 0, 0);
    }
    const int col = col0 + lr;
    if (col < C) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + lk + 4 * q;
        if (i < n) B.M[(size_t)col * ldm + i] -= d[q];
      }
    }
  }
}

__global__ __launch_bounds__(256) void blk_store(const BlkArgs a) {
  const ReduceJob& job = a.job[blockIdx.z];
  const Blk B(job);
  const int n = B.n, m = B.m, p = B.p, ldm = B.L.ldm;
  const ReducedModel& o = job.out;
  const size_t gsz = (size_t)gridDim.x * 256, t0 = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t nh = (size_t)hlen(n);
  for (size_t idx = t0; idx < nh; idx += gsz) {
    // column j of the packed H holds rows 0 .. min(j+1, n-1)
    int j = (int)((sqrt(8.0 * (double)idx + 9.0) - 3.0) * 0.5);
    while (j > 0 && hoff(j) > (int64_t)idx) --j;
    while (j + 1 < n && hoff(j + 1) <= (int64_t)idx) ++j;
    const int i = (int)((int64_t)idx - hoff(j));
    const double x = B.M[(size_t)j * ldm + i];
    o.H[idx] = x;
    o.H32[idx] = (float)x;
  }
  for (size_t idx = t0; idx < (size_t)n * m; idx += gsz) {
    const int i = (int)(idx / m), jj = (int)(idx % m);
    const double x = B.M[(size_t)(n + jj) * ldm + i];
    o.Bt[idx] = x;
    o.Bt32[idx] = (float)x;
  }
  for (size_t idx = t0; idx < (size_t)n * p; idx += gsz) {
    const int i = (int)(idx / p), aa = (int)(idx % p);
    const double x = B.M[(size_t)i * ldm + n + aa];
    o.Ct[idx] = x;
    o.Ct32[idx] = (float)x;
  }
  const ModelIn in(job);
  for (size_t idx = t0; idx < (size_t)p * m; idx += gsz) o.D[idx] = in.d((int)(idx / m), (int)(idx % m));
}

}  // namespace

size_t reduce_blocked_work_bytes(int n, int m, int p) { return blk_layout(n, m, p).total * sizeof(double); }

hipError_t launch_reduce_blocked(const ReduceJob* jobs, int njobs, hipStream_t s) {
  for (int g0 = 0; g0 < njobs; g0 += kBlkBatch) {
    const int nj = std::min(kBlkBatch, njobs - g0);
    BlkArgs a{};
    int nmax = 0, ldm_max = 0, nrb_max = 0;
    size_t load_max = 0, store_max = 0;
    for (int z = 0; z < nj; ++z) {
      const ReduceJob& job = jobs[g0 + z];
      const int n = job.out.n, m = job.out.m, p = job.out.p;
      if (n > kMaxReduceN || !job.work) return hipErrorInvalidValue;
      a.job[z] = job;
      const BlkLayout Lo = blk_layout(n, m, p);
      nmax = std::max(nmax, n);
      ldm_max = std::max(ldm_max, Lo.ldm);
      nrb_max = std::max(nrb_max, Lo.nrb);
      load_max = std::max(load_max, ((size_t)Lo.ldm * (n + m) + 255) / 256);
      store_max = std::max(store_max, ((size_t)hlen(n) + 255) / 256);
    }
    const unsigned Z = (unsigned)nj;
    blk_load<<<dim3((unsigned)std::min<size_t>(2048, load_max), 1, Z), 256, 0, s>>>(a);
    for (int k = 0; k + 2 < nmax; k += kNB) {
      a.k = k;
      int nbk_max = 0, rcols = 0, lcols = 0;
      for (int z = 0; z < nj; ++z) {
        const int n = a.job[z].out.n, nbk = blk_nbk(n, k);
        if (nbk <= 0) continue;
        nbk_max = std::max(nbk_max, nbk);
        rcols = std::max(rcols, n - (k + nbk));                   // right: columns k+nbk .. n-1
        lcols = std::max(lcols, n + a.job[z].out.m - (k + nbk));  // left: .. n+m-1
      }
      for (int j = 0; j < nbk_max; ++j) {
        a.j = j;
        blk_panel<<<dim3(1, 1, Z), kPThreads, 0, s>>>(a);
        blk_rows<<<dim3((unsigned)nrb_max, 1, Z), 256, 0, s>>>(a);
      }
      if (rcols > 0)
        blk_right<<<dim3((unsigned)(ldm_max / kRowBlock), (unsigned)((rcols + 63) / 64), Z), 256, 0, s>>>(a);
      if (lcols > 0) blk_left<<<dim3((unsigned)((lcols + kLeftCols - 1) / kLeftCols), 1, Z), 256, 0, s>>>(a);
    }
    blk_store<<<dim3((unsigned)std::min<size_t>(1024, store_max), 1, Z), 256, 0, s>>>(a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lti
