// lti_freqresp_eval_noalloc: one device-memory request evaluated with no
// allocation at all.  Every buffer the kernels need beyond the caller's
// inputs and outputs -- the reduced model, the reduction's working matrix,
// the refinement queue, merged point records, the reduction job table --
// lives in one file-scope device array, `scratch`, of kNoAllocScratchBytes.
// Each device holds its own copy of that array; its device address is looked
// up once per device (hipGetSymbolAddress) and only that address is handed to
// kernels and copies.  The same kernels as the context path run, in the same
// order: clear the queue counter (and the merged records), reduce, sweep,
// refine queued points.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "lti_freqresp.h"
#include "lti_kernels.h"

namespace lti {
namespace {

// Limits of the scratch-only entry point (see lti_freqresp_eval_noalloc in
// the public header): nx <= 256 (the register and single-workgroup
// reductions), n_omega * min(nu, ny) <= kNoAllocMaxPointCols.
constexpr int kNoAllocMaxN = 256;
constexpr int64_t kNoAllocMaxPointCols = int64_t(1) << 18;
constexpr int64_t kNoAllocMaxPoints = int64_t(1) << 18;
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
constexpr int kNoAllocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_mu;
void* g_scratch[kNoAllocMaxDevices] = {};

size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Device address of this device's copy of `scratch` (the current device).
hipError_t scratch_ptr(int dev, void** out) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

// The reduction kernels read their jobs from a table in device memory: one
// thread writes the job, passed by value, into its slot in scratch (a
// kernel, so that the entry point records no host-to-device copy).
__global__ void put_job_kernel(const ReduceJob job, ReduceJob* dst) { *dst = job; }

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace
}  // namespace lti

using namespace lti;

extern "C" int lti_freqresp_eval_noalloc(int32_t device, const lti_request* q, void* stream) {
  if (!q) return LTI_EINVAL;
  if (q->mem != LTI_MEM_DEVICE) return LTI_EINVAL;
  if (q->nx <= 0 || q->nu <= 0 || q->ny <= 0 || q->n_omega <= 0) return LTI_EINVAL;
  if (!q->A || !q->B || !q->C || !q->omega || !q->G_out) return LTI_EINVAL;
  if (q->precision != LTI_PREC_FP64 && q->precision != LTI_PREC_REFINED) return LTI_EINVAL;
  if (q->points != LTI_POINTS_JW && q->points != LTI_POINTS_S && q->points != LTI_POINTS_Z) return LTI_EINVAL;
  if (q->rtol != q->rtol || q->rtol >= 1.0) return LTI_EINVAL;
  if (q->E) return LTI_EUNSUPPORTED;  // descriptor systems: context path only
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess) return LTI_EDEVICE;
  if (device < 0 || device >= ndev || device >= kNoAllocMaxDevices) return LTI_EINVAL;
  const int n = q->nx, m = q->nu, p = q->ny;
  if (n > kNoAllocMaxN || m > kMaxRhs || p > kMaxRhs) return LTI_EUNSUPPORTED;
  const int trans = p < m ? 1 : 0;
  const int sm = trans ? p : m, sp = trans ? m : p;
  const int64_t K = q->n_omega;
  if (K > kNoAllocMaxPoints || K * sm > kNoAllocMaxPointCols) return LTI_EUNSUPPORTED;
  const int precision = q->dG_out ? LTI_PREC_FP64 : q->precision;
  const double rtol = q->rtol <= 0.0 ? 1e-10 : q->rtol;

  // scratch layout: reduced model | reduction work | job | queue | records
  const size_t b_model = a256(reduced_bytes(n, sm, sp));
  const size_t b_work = a256(reduce_work_bytes(n, sm, sp));
  const size_t b_job = a256(sizeof(ReduceJob));
  const size_t b_queue = a256(8 + 8 * (size_t)K * sm);
  const size_t b_info = q->info_out ? 0 : a256(sizeof(lti_point_info) * (size_t)K);
  if (b_model + b_work + b_job + b_queue + b_info > kNoAllocScratchBytes) return LTI_EUNSUPPORTED;

  DeviceGuard dg(device);
  void* base = nullptr;
  if (scratch_ptr(device, &base) != hipSuccess) return LTI_EDEVICE;
  char* b = static_cast<char*>(base);
  ReducedModel rm;
  reduced_layout(b, n, sm, sp, trans, &rm);
  b += b_model;
  double* work = b_work ? reinterpret_cast<double*>(b) : nullptr;
  b += b_work;
  ReduceJob* djob = reinterpret_cast<ReduceJob*>(b);
  b += b_job;
  uint32_t* fbq = reinterpret_cast<uint32_t*>(b);
  b += b_queue;
  lti_point_info* info = q->info_out ? q->info_out : reinterpret_cast<lti_point_info*>(b);

  const hipStream_t s = static_cast<hipStream_t>(stream);
  ReqDesc desc{};
  desc.H = rm.H;
  desc.Bt = rm.Bt;
  desc.Ct = rm.Ct;
  desc.D = rm.D;
  desc.H32 = rm.H32;
  desc.Bt32 = rm.Bt32;
  desc.Ct32 = rm.Ct32;
  desc.omega = q->omega;
  desc.G = q->G_out;
  desc.dG = q->dG_out;
  desc.info = info;
  desc.fbq = fbq;
  desc.n = n;
  desc.m = sm;
  desc.p = sp;
  desc.precision = precision;
  desc.rtol = rtol;
  desc.flags = (trans ? kFlagTrans : 0u) | ((uint32_t)q->points << 8);

  // the tiling an idle context would choose for this request alone
  TileKnobs kn;
  const TilePlan tp = plan_tiles(precision, n, sm, sp, K, kTargetTilesFour, kTargetTilesOne, kn);
  if (tp.kclass < 0 || tp.ntiles <= 0 || tp.ntiles > (int64_t)INT32_MAX) return LTI_EUNSUPPORTED;
  if (tp.S > 1) desc.flags |= kFlagMergeInfo;

  // every call shares this device's scratch: clear what must start at zero
  ZeroLaunch Z{};
  Z.n = 1;
  Z.e[0].p = fbq;
  Z.e[0].words = 1u;
  if (tp.S > 1) {
    Z.n = 2;
    Z.e[1].p = reinterpret_cast<uint32_t*>(info);
    Z.e[1].words = (uint32_t)(2 * K);
  }
  hipError_t e = launch_zero(Z, s);

  ReduceJob job{};
  job.A = q->A;
  job.B = q->B;
  job.C = q->C;
  job.D = q->D;
  job.out = rm;
  job.work = work;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(put_job_kernel, dim3(1), dim3(1), 0, s, job, djob);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    ReduceLaunch RL;
    RL.jobs = djob;
    RL.host_jobs = &job;
    RL.njobs = 1;
    e = launch_reduce(RL, reduce_class(n, sm, sp), s);
  }
  if (e == hipSuccess) {
    SweepLaunch L;
    L.nseg = 1;
    L.ntiles = (int)tp.ntiles;
    SweepSeg& sg = L.seg[0];
    sg.rd = desc;
    sg.tile0 = 0;
    sg.first = 0;
    sg.K = (uint32_t)K;
    sg.F = (uint16_t)tp.F;
    sg.S = (uint8_t)tp.S;
    sg.mc = (uint8_t)tp.mc;
    e = launch_any_sweep(tp.kclass, L, tp.stage, s);
  }
  if (e == hipSuccess) {
    DDLaunch D;
    D.nseg = 1;
    D.seg[0].rd = desc;
    D.seg[0].rm = rm;
    D.seg[0].K = (uint64_t)K;
    const int grid = (int)std::max<int64_t>(16, std::min<int64_t>(1024, K * tp.S / 32));
    e = launch_refine_dd(D, grid, s);
  }
  return e == hipSuccess ? LTI_OK : LTI_EDEVICE;
}
