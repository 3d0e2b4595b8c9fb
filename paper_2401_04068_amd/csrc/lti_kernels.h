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

// The resident reduced model of one state-space system, all in one arena
// block.  H = Q^T A Q (packed), Bt = Q^T B (n x m row-major), Ct = (C Q)^T
// (n x p row-major, so row i holds column i of C Q), D (p x m row-major),
// plus float32 copies of H, Bt and Ct for the refined path.
struct ReducedModel {
  double* H;
  double* Bt;
  double* Ct;
  double* D;
  float* H32;
  float* Bt32;
  float* Ct32;
  int n, m, p, pad;
};

size_t reduced_bytes(int n, int m, int p);
void reduced_layout(void* base, int n, int m, int p, ReducedModel* out);

// One reduction job: read A, B, C, D (device pointers, row-major; D may be
// null), write the reduced model.  `work` is a scratch area of
// reduce_work_bytes(n, m, p) bytes (null for the register kernel).
struct ReduceJob {
  const double* A;
  const double* B;
  const double* C;
  const double* D;
  ReducedModel out;
  double* work;
};

constexpr int kMaxReduceN = 1024;
// Reduction kernel classes: 0 .. kNumRegClasses-1 keep the working matrix in
// registers (class S-1 for S = ceil(max(n+p, n+m) / 16) <= 9, n <= 128);
// kReduceGlobal keeps it in a global scratch area (one workgroup per model);
// kReduceBlocked runs the blocked reduction over the whole GPU, one model at a
// time (reduce_blocked.hip).
constexpr int kMaxRegReduceN = 128;
constexpr int kNumRegClasses = 9;
constexpr int kReduceGlobal = kNumRegClasses;       // 128 < n <= kMaxGlobalReduceN
constexpr int kReduceBlocked = kNumRegClasses + 1;  // larger n: blocked, whole GPU
constexpr int kNumReduceClasses = kNumRegClasses + 2;
constexpr int kMaxGlobalReduceN = 256;
int reduce_class(int n, int m, int p);
// Global scratch bytes a job of this shape needs (0 for register classes).
size_t reduce_work_bytes(int n, int m, int p);
size_t reduce_blocked_work_bytes(int n, int m, int p);
hipError_t launch_reduce_blocked(const ReduceJob& job, hipStream_t s);
// Up to kMaxInlineJobs reduction jobs of one class, passed to the kernel by
// value; one workgroup per job.
constexpr int kMaxInlineJobs = 24;
struct ReduceLaunch {
  int njobs;
  ReduceJob job[kMaxInlineJobs];
};
static_assert(sizeof(ReduceLaunch) <= 3072, "reduction launch arguments must stay small");
hipError_t launch_reduce(const ReduceLaunch& L, int rclass, hipStream_t s);

// Per-request descriptor, handed to the sweep kernels in their launch
// arguments.
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
  lti_point_info* info;
  int n, m, p, precision;
  double rtol;
};

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
static_assert(sizeof(SweepLaunch) <= 2048, "sweep launch arguments must stay small");

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

// Workgroup-per-frequency kernels (sweepwg.hip): float64 path, 256 < n <= 1024,
// at most 4 right-hand-side columns per tile; -1 when not covered.
constexpr int kMaxNWG = 1024;
constexpr int kNumSweepWGClasses = 3;
int sweep_wg_class(int precision, int n, int mc);
hipError_t launch_sweep_wg(int cls, const SweepLaunch& L, hipStream_t s);

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

}  // namespace lti
