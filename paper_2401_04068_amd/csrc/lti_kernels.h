// Internal interface between the runtime (runtime.cpp) and the HIP kernels
// (reduce.hip, sweep.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lti_freqresp.h"

namespace lti {

// Packed column-major upper Hessenberg storage: column j holds rows
// 0 .. min(j+1, n-1), so column j starts at j(j+3)/2 and the whole matrix
// takes (n-1)(n+2)/2 + n entries.
__host__ __device__ inline int64_t hoff(int j) { return (int64_t)j * (j + 3) / 2; }
__host__ __device__ inline int64_t hlen(int n) { return (int64_t)(n - 1) * (n + 2) / 2 + n; }

// Reflector storage of a reduction: reflector k (k = 0 .. n-3) is
// P_k = I - tau_k v v^T with v = e_{k+1} + (entries k+2 .. n-1), and those
// entries are kept at V[voff(n, k) + (i - k - 2)], so that Q = P_0 P_1 ...
// P_{n-3} can be applied to vectors afterwards.
__host__ __device__ inline int64_t voff(int n, int k) { return (int64_t)k * (n - 2) - (int64_t)k * (k - 1) / 2; }
__host__ __device__ inline int64_t vlen(int n) { return n >= 3 ? (int64_t)(n - 2) * (n - 1) / 2 : 0; }

// The resident reduced model of one state-space system, all in one arena
// block.  H = Q^T A Q (packed), Bt = Q^T B (n x m row-major), Ct = (C Q)^T
// (n x p row-major, so row i holds column i of C Q), D (p x m row-major),
// plus float32 copies of H, Bt and Ct for the refined path.  The solved
// system is (A, B, C, D) itself, or (A^T, C^T, B^T, D^T) when `trans` is set
// (fewer outputs than inputs: G^T of the transposed system needs only
// min(nu, ny) right-hand sides); n, m, p are the solved system's sizes.  A0,
// B0, C0 hold that system as given (row-major, float64) and V, tau the
// reflectors, for the extended-precision refinement of ill-conditioned points.
struct ReducedModel {
  double* H;
  double* Bt;
  double* Ct;
  double* D;
  float* H32;
  float* Bt32;
  float* Ct32;
  double* A0;
  double* B0;
  double* C0;
  double* V;
  double* tau;
  double* T;  // descriptor systems: Q^T E Z, packed upper triangular (column
              // j holds rows 0 .. j, from j (j + 1) / 2); null otherwise
  int n, m, p, trans;
};

// desc: the model is a descriptor system (T is stored).
size_t reduced_bytes(int n, int m, int p, bool desc = false);
void reduced_layout(void* base, int n, int m, int p, int trans, ReducedModel* out, bool desc = false);

// One reduction job: read A, B, C, D (device pointers, row-major, the
// request's own sizes; D may be null), write the reduced model (out.trans
// says whether the transposed system is reduced).  `work` is a scratch area
// of reduce_work_bytes(n, m, p) bytes (null for the register kernel).
struct ReduceJob {
  const double* A;
  const double* B;
  const double* C;
  const double* D;
  const double* E;  // descriptor systems only (row-major n x n), else null
  ReducedModel out;
  double* work;
};

// Entry (i, j) of the solved system's matrices, read from the request's
// arrays (n, m, p: the solved system's sizes).
struct ModelIn {
  const double *A, *B, *C, *D, *E;
  int n, m, p, trans;
  __host__ __device__ ModelIn(const ReduceJob& j)
      : A(j.A), B(j.B), C(j.C), D(j.D), E(j.E), n(j.out.n), m(j.out.m), p(j.out.p), trans(j.out.trans) {}
  __host__ __device__ double e(int i, int k) const {
    return trans ? E[(size_t)k * n + i] : E[(size_t)i * n + k];
  }
  __host__ __device__ double a(int i, int k) const {
    return trans ? A[(size_t)k * n + i] : A[(size_t)i * n + k];
  }
  __host__ __device__ double b(int i, int c) const {
    return trans ? C[(size_t)c * n + i] : B[(size_t)i * m + c];
  }
  __host__ __device__ double c(int r, int k) const {
    return trans ? B[(size_t)k * p + r] : C[(size_t)r * n + k];
  }
  __host__ __device__ double d(int r, int c) const {
    return !D ? 0.0 : trans ? D[(size_t)c * p + r] : D[(size_t)r * m + c];
  }
};

constexpr int kMaxReduceN = 1024;
// Reduction kernel classes: 0 .. kNumRegClasses-1 keep the working matrix in
// registers (class S-1 for S = ceil(max(n+p, n+m) / 16) <= 9, n <= 128);
// kReduceGlobal keeps it in a global scratch area (one workgroup per model);
// kReduceBlocked runs the blocked reduction over the whole GPU, up to eight
// models in each launch of its kernel sequence (reduce_blocked.hip).
constexpr int kMaxRegReduceN = 128;
constexpr int kNumRegClasses = 9;
constexpr int kReduceGlobal = kNumRegClasses;       // 128 < n <= kMaxGlobalReduceN
constexpr int kReduceBlocked = kNumRegClasses + 1;  // larger n: blocked, whole GPU
// Descriptor systems (n <= kMaxN): Hessenberg-triangular reduction, one
// workgroup per model (reduce_ht.hip).
constexpr int kReduceHT = kNumRegClasses + 2;
constexpr int kNumReduceClasses = kNumRegClasses + 3;
size_t reduce_ht_work_bytes(int n, int m, int p);
hipError_t launch_reduce_ht(const struct ReduceLaunch& L, hipStream_t s);
constexpr int kMaxGlobalReduceN = 256;
int reduce_class(int n, int m, int p);
// Global scratch bytes a job of this shape needs (0 for register classes).
size_t reduce_work_bytes(int n, int m, int p);
size_t reduce_blocked_work_bytes(int n, int m, int p);
hipError_t launch_reduce_blocked(const ReduceJob* jobs, int njobs, hipStream_t s);
// The reduction jobs of one class in one launch, one workgroup per job (the
// blocked class: one kernel sequence per eight jobs): `jobs` is a table in device
// memory, uploaded with the pass that queued them.  `host_jobs` is the same
// table in host memory (the blocked class reads its jobs from there).
struct ReduceLaunch {
  const ReduceJob* jobs;
  const ReduceJob* host_jobs;
  int njobs;
};
hipError_t launch_reduce(const ReduceLaunch& L, int rclass, hipStream_t s);

// Clear up to kMaxZero device ranges (32-bit words), one workgroup each: the
// refinement queue counters and merged point records of newly admitted
// requests.  A kernel, not hipMemsetAsync, so that a captured stream replays
// it faithfully.
constexpr int kMaxZero = 64;
struct ZeroLaunch {
  int n;
  struct {
    uint32_t* p;
    uint32_t words;
  } e[kMaxZero];
};
hipError_t launch_zero(const ZeroLaunch& Z, hipStream_t s);

// Summaries of the point records of the requests a sweep batch finishes,
// one workgroup per request: points per path code and the largest error
// estimate, so that the host reads 64 bytes per request instead of every
// record.  `tab` and `out` are device arrays of n entries.
struct FinEntry {
  const lti_point_info* info;
  uint64_t K;
};
struct PointSummary {
  uint32_t count[8];  // points per LTI_PATH_* code (codes 0-7)
  float max_est;      // largest est_rel_err (NaN records ignored)
  uint32_t pad[7];
};
static_assert(sizeof(PointSummary) == 64, "summary records are 64 bytes");
hipError_t launch_summarize(const FinEntry* tab, PointSummary* out, int n, hipStream_t s);

// Per-request descriptor, handed to the sweep kernels in their launch
// arguments.
//
// Evaluation points (flags bits 8-9): kPointsJW, s_k = j omega[k];
// kPointsS, s_k = omega[2k] + j omega[2k+1]; kPointsZ, the discrete-time
// point z_k = exp(j omega[k]) (omega[k] in radians per sample).  Every
// kernel solves (s_k I - H) X = Q^T B.
//
// Points whose solve cannot be trusted in the kernel's own precision (a
// refined point whose iteration stalled, a float64 point whose estimated
// error exceeds rtol) are not written by the sweep: they are appended to the
// request's queue `fbq` (fbq[0] = count, entry e at fbq[2 + 2e]: the point
// index, then first column | columns << 8 | float32 solves << 16 | reason
// << 24) and finished by the extended-precision refinement kernel.
constexpr uint32_t kFlagTrans = 1u;      // G^T of the transposed system
constexpr uint32_t kFlagMergeInfo = 2u;  // columns split over tiles: info merged with atomic max
constexpr uint32_t kFlagForceDD = 4u;    // every point takes the extended refinement (testing)
constexpr uint32_t kFlagDescriptor = 8u; // descriptor system: M = s T - H, never queued
constexpr int kPointsJW = 0, kPointsS = 1, kPointsZ = 2;
constexpr int kReasonFP64 = 0, kReasonStall = 1;
struct ReqDesc {
  const double* H;
  const double* Bt;
  const double* Ct;
  const double* D;
  const float* H32;
  const float* Bt32;
  const float* Ct32;
  const double* omega;
  double* G;
  double* dG;  // dG/ds (float64 path only), or null
  const double* T;  // descriptor systems: packed upper triangular Q^T E Z, else null
  lti_point_info* info;
  uint32_t* fbq;
  int n, m, p, precision;
  double rtol;
  uint32_t flags;
  uint32_t pad;
};

// Output index of G(a, j) (rows a < p, columns j < m of the solved system)
// within one point's p x m block of the caller's [k][row][column] layout.
__host__ __device__ inline int g_index(const ReqDesc& rd, int a, int j) {
  return (rd.flags & kFlagTrans) ? j * rd.p + a : a * rd.m + j;
}

// A sweep launch covers tiles of up to kMaxSegs requests and is passed to the
// kernel by value (kernel arguments: no copy, no descriptor in memory).
// Tile t of a request holds frequencies [F (t / S), F (t / S) + F) (clipped
// to K) and right-hand-side columns [mc (t % S), mc (t % S) + mc) (clipped to
// m); segment s gives launch tiles [tile0, next segment's tile0) to the
// request's tiles first, first + 1, ...
struct SweepSeg {
  ReqDesc rd;
  uint32_t tile0;
  uint32_t first;
  uint32_t K;
  uint16_t F;
  uint8_t S;
  uint8_t mc;
};
constexpr int kMaxSegs = 16;
struct SweepLaunch {
  int nseg;
  int ntiles;
  SweepSeg seg[kMaxSegs];
};
static_assert(sizeof(SweepLaunch) <= 3072, "sweep launch arguments must stay small");

// Sweep kernel classes: precision x rows-per-lane (1, 2, 4 -> n <= 64, 128,
// 256) x right-hand-side capacity (1, 2, 4, 8, 16).
constexpr int kNumRowClasses = 3;
constexpr int kNumRhsClasses = 5;
constexpr int kNumSweepClasses = 2 * kNumRowClasses * kNumRhsClasses;
constexpr int kMaxN = 256;
constexpr int kMaxRhs = 16;
int sweep_class(int precision, int n, int m);

// Four-frequencies-per-wavefront kernels (sweep16.hip), both precisions,
// n <= 64 and at most 4 right-hand-side columns per tile; -1 when the request
// is not covered.  Their tiles should hold a multiple of 4 frequencies.
constexpr int kNumSweep16Classes = 18;
int sweep16_class(int precision, int n, int mc);
hipError_t launch_sweep16(int cls, const SweepLaunch& L, hipStream_t s);

// Two-frequencies-per-wavefront kernels (sweep16.hip, 32-lane groups), both
// precisions, 64 < n <= 128 and at most 4 right-hand-side columns per tile;
// -1 when not covered.  Their tiles should hold a multiple of 2 frequencies.
constexpr int kNumSweep32Classes = 12;
int sweep32_class(int precision, int n, int mc);
hipError_t launch_sweep32(int cls, const SweepLaunch& L, hipStream_t s);

// Workgroup-per-frequency kernels (sweepwg.hip): both precisions,
// 256 < n <= 1024, at most 4 right-hand-side columns per tile; -1 when not
// covered.
constexpr int kMaxNWG = 1024;
constexpr int kNumSweepWGClasses = 6;
int sweep_wg_class(int precision, int n, int mc);
hipError_t launch_sweep_wg(int cls, const SweepLaunch& L, hipStream_t s);

// Extended-precision refinement (sweepwg.hip) of the points the sweeps of a
// request queued (ReqDesc.fbq), after all of the request's sweep tiles: one
// workgroup per queued entry at a time, `grid` workgroups in all.
constexpr int kMaxDDSegs = 11;
struct DDSeg {
  ReqDesc rd;
  ReducedModel rm;
  uint64_t K;  // points of the request (bounds the queue)
};
struct DDLaunch {
  int nseg;
  DDSeg seg[kMaxDDSegs];
};
static_assert(sizeof(DDLaunch) <= 3072, "refinement launch arguments must stay small");
hipError_t launch_refine_dd(const DDLaunch& L, int grid, hipStream_t s);

// LDS staging of one request's reduced model by a sweep workgroup: H, Bt and
// Ct in float64, plus H and Bt in float32 for the refined path, each block
// 16-byte aligned, in that order.  A workgroup stages when its four tiles
// belong to one request and the model fits in kStageLimit bytes; otherwise
// it reads the model from global memory.
constexpr size_t kStageLimit = 64 * 1024;
struct StageLayout {
  size_t H, Bt, Ct, H32, Bt32, bytes;
};
__host__ __device__ inline size_t stage_align(size_t x) { return (x + 15) & ~size_t(15); }
__host__ __device__ inline StageLayout stage_layout(int precision, int n, int m, int p) {
  StageLayout L;
  const size_t hl = (size_t)hlen(n);
  size_t o = 0;
  L.H = o;
  o += stage_align(hl * 8);
  L.Bt = o;
  o += stage_align((size_t)n * m * 8);
  L.Ct = o;
  o += stage_align((size_t)n * p * 8);
  L.H32 = o;
  L.Bt32 = o;
  if (precision == LTI_PREC_REFINED) {
    o += stage_align(hl * 4);
    L.Bt32 = o;
    o += stage_align((size_t)n * m * 4);
  }
  L.bytes = o;
  return L;
}
// Staging bytes of a request, 0 when it does not fit kStageLimit.
__host__ __device__ inline size_t stage_bytes(int precision, int n, int m, int p) {
  const size_t b = stage_layout(precision, n, m, p).bytes;
  return b <= kStageLimit ? b : 0;
}
// lds_bytes: dynamic LDS for staging (the largest stage_bytes() of the
// launch's requests; 0 disables staging).
hipError_t launch_sweep(int kclass, const SweepLaunch& L, size_t lds_bytes, hipStream_t s);

// Descriptor systems, float64, n <= kMaxN: one frequency per wavefront with
// M = s T - H (sweep.hip); classes as sweep_class(LTI_PREC_FP64, n, m).
constexpr int kNumSweepDescClasses = kNumRowClasses * kNumRhsClasses;
hipError_t launch_sweep_desc(int kclass, const SweepLaunch& L, hipStream_t s);

// All sweep kernel classes in one index space: [0, kNumSweepClasses) one
// frequency per wavefront, then the four-frequency classes, then the
// workgroup classes, then the descriptor classes, then the two-frequency
// classes.
constexpr int kSweepDescBase = kNumSweepClasses + kNumSweep16Classes + kNumSweepWGClasses;
constexpr int kSweep32Base = kSweepDescBase + kNumSweepDescClasses;
constexpr int kAllSweepClasses = kSweep32Base + kNumSweep32Classes;
hipError_t launch_any_sweep(int kclass, const SweepLaunch& L, size_t lds_bytes, hipStream_t s);

// How a request's solves are cut into tiles (runtime.cpp): F frequencies
// per tile, its m right-hand-side columns in S groups of mc, the kernel
// class, and the waves each tile occupies.  `avail_waves`: wavefronts the
// device can still take before splitting columns stops paying (columns are
// split only while the request alone would leave the device short).
struct TilePlan {
  int kclass, F, S, mc, waves_per_tile;
  int64_t ntiles;
  size_t stage;
};
// Wavefronts a request alone should offer before its right-hand-side
// columns stop being split over tiles, on an otherwise idle device: 256 CUs
// x 4 SIMDs x 4 resident waves for one-frequency tiles, a quarter of that for
// four-frequency tiles (each already carries four solves); two-frequency
// tiles take half of the one-frequency figure.
constexpr int64_t kTargetTilesOne = 4096;
constexpr int64_t kTargetTilesFour = 1024;
struct TileKnobs {
  int tile_points = 0;   // 0: automatic
  int rhs_split = 0;     // 0: automatic
  bool use_sweep16 = true;
  bool use_sweep32 = true;
  int sweep32_max_cols = kMaxRhs;  // widest request (min(m, p)) sent to the two-frequency kernels
  bool descriptor = false;  // descriptor system: float64 one-frequency kernels only
};
TilePlan plan_tiles(int precision, int n, int sm, int sp, int64_t K, int64_t avail_waves4, int64_t avail_waves1,
                    const TileKnobs& kn);

}  // namespace lti
