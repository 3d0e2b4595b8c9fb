// Serving runtime behind the C ABI: arena sub-allocation, resident reduced
// models, admission by memory budget, and continuous batching of the
// per-frequency solves of every live request into shared kernel launches.
//
// Device work is issued on two streams by a scheduling pass
// (pump) that runs under the context lock: on the context's scheduler thread,
// and inline on the caller's thread in submit() and in a waiting poll(), so a
// lone request starts and completes without a thread hand-off.  A pass:
//
//   admit    pending requests in arrival order while their memory fits:
//            upload inputs, reuse a resident reduced model or queue a
//            reduction job (the jobs of one pass share a launch per kernel
//            class).  Uploads and reductions go to an idle one of
//            kAdmitStreams admission streams and end with an event that the
//            requests of the pass (and the models it reduced) keep; a sweep
//            launch first waits on the events of its requests, so reductions
//            run beside sweeps.  While every admission stream is still busy,
//            new requests wait, and are then admitted together: their
//            reductions share launches and run side by side (one reduction
//            occupies a single CU);
//   launch   gather up to max_batch_tiles tiles from the live requests
//            (oldest first), group them by kernel class and launch on the
//            sweep stream; at most kInflight batches are outstanding, so
//            requests that arrive meanwhile join the next batch;
//   retire   when a batch's event has fired, credit its tiles; a request
//            whose tiles are all done gets its D2H copy and then becomes
//            visible to poll().
//
// Host inputs are copied at submit() into pinned staging owned by the
// library, so every H2D and D2H copy is a true asynchronous DMA that never
// stalls the scheduler behind queued kernels.  The descriptors the kernels
// need (reduction jobs, per-request descriptors and tile ranges) travel in
// the kernel arguments: nothing but the inputs and results is ever copied.
#include <hip/hip_runtime.h>
#include <sys/prctl.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lti_freqresp.h"
#include "lti_kernels.h"

namespace lti {
namespace {

constexpr size_t kAlign = 256;
// Sweep batches outstanding: one.  A new batch is formed when the previous
// one completes, so requests admitted meanwhile share it (bigger launches,
// and new requests wait behind one batch instead of a queue of them); this
// measured best for throughput and for serving latency.
constexpr int kInflight = 1;
// Streams: one admission stream and one sweep stream by default (a process
// gets few hardware queues, four by default, and streams that share one run
// in order).  With one admission stream, requests that arrive during a
// reduction are admitted together afterwards, so their reductions and their
// sweeps share launches; more streams (a tuning knob) measured slower.
constexpr int kAdmitStreams = 2;
constexpr int kSweepStreams = 2;
// Reduction jobs queued by one admission pass (bounds one pass's work).
constexpr int kMaxJobs = 1024;
constexpr int kDefaultMaxPending = 8192;
constexpr int kDefaultBatchTiles = 16384;
constexpr size_t kDefaultStaging = size_t(256) << 20;
// A waiting poll() runs scheduling passes itself for up to this long.
constexpr int64_t kPollSpinUs = 2000;
// The scheduler thread backs off while a caller's thread has run a
// scheduling pass within this window.
constexpr double kClientActiveUs = 200.0;
// Tiles (wavefronts) one request should offer before its columns are split:
// 256 CUs x 4 SIMDs x 4 resident waves.
constexpr int64_t kTargetTiles = 4096;
// The same for four-frequency tiles (each already carries four solves).
constexpr int64_t kTargetTiles16 = 1024;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

using Clock = std::chrono::steady_clock;

// First-fit allocator over a fixed range with coalescing frees.
class Arena {
 public:
  void init(char* base, size_t size) {
    base_ = base;
    size_ = size;
    free_.clear();
    if (size) free_[0] = size;
    used_ = peak_ = 0;
  }
  void* alloc(size_t bytes) {
    bytes = align_up(std::max<size_t>(bytes, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        const size_t off = it->first;
        const size_t rest = it->second - bytes;
        free_.erase(it);
        if (rest) free_[off + bytes] = rest;
        used_ += bytes;
        peak_ = std::max(peak_, used_);
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(void* p, size_t bytes) {
    if (!p) return;
    bytes = align_up(std::max<size_t>(bytes, 1));
    const size_t off = static_cast<char*>(p) - base_;
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  bool can_ever_fit(size_t bytes) const { return align_up(bytes) <= size_; }
  size_t size() const { return size_; }
  size_t used() const { return used_; }
  size_t peak() const { return peak_; }

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;
  size_t used_ = 0, peak_ = 0;
};

// The end of one admission pass on its stream (uploads and reductions),
// shared by the requests admitted in it and by the models it reduced.
struct PassEvent {
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;  // where the pass was issued
  int refs = 0;
};

struct Resident {
  PassEvent* ready = nullptr;  // pass that reduced it, until a user completed
  uint64_t key = 0;
  uint64_t hash = 0;
  int n = 0, m = 0, p = 0;
  void* block = nullptr;
  size_t bytes = 0;
  ReducedModel rm{};
  int refs = 0;
  uint64_t last_use = 0;
};

enum class RState { kPending, kLive, kFinishing, kDone, kFailed };

// Host-side staging of a host-memory request: A, B, C, D, omega and (at
// completion) G and info, in one pinned block when the pool has room.
struct HostStage {
  char* base = nullptr;  // pinned block, or fallback.data()
  size_t bytes = 0;
  bool pinned = false;
  std::vector<char> fallback;
  size_t offA = 0, offB = 0, offC = 0, offD = 0, offW = 0, offG = 0, offInfo = 0;
};

struct Request {
  uint64_t id = 0;
  lti_request req{};
  RState state = RState::kPending;
  int status = LTI_OK;
  uint64_t hash = 0;
  HostStage hs;
  Resident* model = nullptr;
  bool reused = false;
  PassEvent* ready = nullptr;        // its own admission pass
  PassEvent* model_ready = nullptr;  // the pass that reduced a reused model
  void* block = nullptr;  // device: A..D, omega, G, info, reduction scratch
  size_t block_bytes = 0;
  size_t dOffG = 0;
  ReqDesc desc{};         // handed to the sweep kernels in their arguments
  int kclass = -1;
  int64_t K = 0;
  int F = 1;        // frequencies per tile
  int S = 1;        // right-hand-side column groups per frequency block
  int mc = 1;       // columns per group
  size_t stage = 0; // LDS bytes a sweep workgroup needs to stage the model
  int64_t ntiles = 0, next_tile = 0, tiles_done = 0;
  int waves_per_tile = 1;
  hipEvent_t d2h_ev = nullptr;
  lti_result res{};
};

struct Batch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  bool timed = false;
  std::vector<std::pair<Request*, int64_t>> credit;
};

struct TimedPair {
  hipEvent_t a, b;
};

// FNV-1a over 64-bit words (the arrays hashed here are doubles), then any
// remaining bytes.
uint64_t fnv1a(const void* data, size_t bytes, uint64_t h) {
  const unsigned char* p = static_cast<const unsigned char*>(data);
  size_t i = 0;
  for (; i + 8 <= bytes; i += 8) {
    uint64_t w;
    std::memcpy(&w, p + i, 8);
    h ^= w;
    h *= 1099511628211ull;
  }
  for (; i < bytes; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

bool all_finite(const double* x, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace
}  // namespace lti

using namespace lti;

struct lti_ctx {
  int device = 0;
  hipStream_t stream = nullptr;               // first sweep stream; result copies
  hipStream_t sstreams[kSweepStreams] = {};  // sweeps ([0] = stream)
  int next_sstream = 0;
  int n_sstreams = 1;
  hipStream_t rstreams[kAdmitStreams] = {};  // uploads and reductions
  int next_rstream = 0;
  int n_rstreams = 1;
  int max_inflight = kInflight;  // sweep batches outstanding
  hipStream_t rstream = nullptr;             // the current pass's stream
  PassEvent* last_pass[kAdmitStreams] = {};  // the last pass on each
  std::atomic<double> client_pump_us{-1e30};  // when a caller's thread last ran a pass
  PassEvent* pass = nullptr;                 // the current pass's event
  std::vector<PassEvent*> pass_events;       // all live ones
  bool own_stream = false;
  uint32_t flags = 0;
  int max_pending = kDefaultMaxPending;
  int tile_points = 0;
  int batch_tiles = kDefaultBatchTiles;
  int rhs_split = 0;        // 0: automatic
  bool stage_lds = true;    // LDS staging of reduced models in the sweep
  bool use_sweep16 = true;  // four-frequencies-per-wavefront kernels where they apply
  int64_t target_tiles16 = kTargetTiles16;
  int64_t target_tiles = kTargetTiles;
  int64_t outstanding_waves = 0;  // waves of admitted tiles not yet retired
  Arena arena;
  Arena staging;  // pinned host pool
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::thread thread;
  bool stop = false;
  bool device_error = false;

  uint64_t next_id = 1;
  uint64_t use_clock = 0;
  std::deque<Request*> pending;
  std::vector<Request*> live;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<std::unique_ptr<Resident>> residents;
  std::deque<Batch> inflight;
  std::deque<TimedPair> reduce_timing;

  char* staging_block = nullptr;  // the pinned allocation behind `staging`
  std::vector<hipEvent_t> event_pool, timing_pool;

  lti_stats stats{};

  double now_us() const {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  }
};

namespace {

hipEvent_t get_event(lti_ctx* c, bool timing) {
  auto& pool = timing ? c->timing_pool : c->event_pool;
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, timing ? hipEventDefault : hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

void put_event(lti_ctx* c, hipEvent_t e, bool timing) {
  if (e) (timing ? c->timing_pool : c->event_pool).push_back(e);
}

PassEvent* pass_ref(PassEvent* pe) {
  if (pe) pe->refs++;
  return pe;
}

void pass_release(lti_ctx* c, PassEvent*& pe) {
  if (!pe) return;
  if (--pe->refs == 0) {
    put_event(c, pe->ev, false);
    c->pass_events.erase(std::find(c->pass_events.begin(), c->pass_events.end(), pe));
    delete pe;
  }
  pe = nullptr;
}

void fail_all(lti_ctx* c, int code) {
  c->device_error = true;
  for (auto& kv : c->all) {
    Request* r = kv.second.get();
    if (r->state != RState::kDone && r->state != RState::kFailed) {
      r->state = RState::kFailed;
      r->status = code;
      r->res.status = code;
      c->stats.requests_failed++;
    }
  }
  c->pending.clear();
  c->live.clear();
  c->cv_done.notify_all();
}

void release_stage(lti_ctx* c, HostStage& hs) {
  if (hs.pinned && hs.base) c->staging.release(hs.base, hs.bytes);
  hs.base = nullptr;
  hs.pinned = false;
  hs.fallback.clear();
  hs.fallback.shrink_to_fit();
}

// Device bytes of a request (besides a shared resident model); the block holds
// [A..D | omega | G | info] (host-memory requests), then the reduction scratch.
struct Need {
  size_t omega = 0, G = 0, info = 0, inputs = 0, work = 0, model = 0;
  size_t block() const { return omega + G + info + inputs + work; }
};

Need request_need(const lti_request& q, bool needs_model) {
  const int n = q.nx, m = q.nu, p = q.ny;
  Need nd;
  if (q.mem == LTI_MEM_HOST) {
    nd.omega = align_up(sizeof(double) * q.n_omega);
    nd.G = align_up(sizeof(double) * 2 * (size_t)q.n_omega * p * m);
    nd.info = q.info_out ? align_up(sizeof(lti_point_info) * q.n_omega) : 0;
  }
  if (needs_model) {
    if (q.mem == LTI_MEM_HOST)  // same per-matrix alignment as the host staging
      nd.inputs = align_up(sizeof(double) * n * n) + align_up(sizeof(double) * n * m) +
                  align_up(sizeof(double) * p * n) + align_up(sizeof(double) * p * m);
    nd.work = reduce_work_bytes(n, m, p);
    nd.model = align_up(reduced_bytes(n, m, p));
  }
  return nd;
}

Resident* find_resident(lti_ctx* c, const Request& r) {
  if (r.req.model_key == 0) return nullptr;
  for (auto& up : c->residents) {
    Resident* res = up.get();
    if (res->key == r.req.model_key && res->n == r.req.nx && res->m == r.req.nu && res->p == r.req.ny &&
        res->hash == r.hash)
      return res;
  }
  return nullptr;
}

void drop_resident(lti_ctx* c, Resident* res) {
  pass_release(c, res->ready);
  c->arena.release(res->block, res->bytes);
  for (auto it = c->residents.begin(); it != c->residents.end(); ++it) {
    if (it->get() == res) {
      c->residents.erase(it);
      return;
    }
  }
}

// Allocate, evicting unreferenced resident models (least recently used
// first) while that helps.
void* alloc_evicting(lti_ctx* c, size_t bytes) {
  void* p = c->arena.alloc(bytes);
  while (!p) {
    Resident* victim = nullptr;
    for (auto& up : c->residents)
      if (up->refs == 0 && (!victim || up->last_use < victim->last_use)) victim = up.get();
    if (!victim) return nullptr;
    drop_resident(c, victim);
    p = c->arena.alloc(bytes);
  }
  return p;
}

void release_request_memory(lti_ctx* c, Request* r) {
  if (r->block) c->arena.release(r->block, r->block_bytes);
  r->block = nullptr;
  pass_release(c, r->ready);
  pass_release(c, r->model_ready);
  if (r->model) {
    Resident* res = r->model;
    // a user of the model has completed, so its reduction has too
    if (r->state == RState::kDone) pass_release(c, res->ready);
    res->refs--;
    r->model = nullptr;
    if (res->key == 0 && res->refs == 0) drop_resident(c, res);
  }
}

// Try to admit one request.  Returns false when it has to wait for memory.
struct JobLists {
  std::vector<ReduceJob> jobs[kNumReduceClasses];
  bool copies = false;  // uploads were issued on the admission stream
  size_t total() const {
    size_t t = 0;
    for (const auto& v : jobs) t += v.size();
    return t;
  }
};

bool admit_one(lti_ctx* c, Request* r, JobLists& jl) {
  const lti_request& q = r->req;
  const int n = q.nx, m = q.nu, p = q.ny;
  Resident* res = find_resident(c, *r);
  const bool needs_model = (res == nullptr);
  if (needs_model && (int)jl.total() >= kMaxJobs) return false;
  const Need nd = request_need(q, needs_model);
  void* mblock = nullptr;
  if (needs_model) {
    mblock = alloc_evicting(c, nd.model);
    if (!mblock) return false;
  }
  void* block = alloc_evicting(c, nd.block());
  if (!block) {
    if (mblock) c->arena.release(mblock, nd.model);
    return false;
  }
  if (needs_model) {
    auto up = std::make_unique<Resident>();
    res = up.get();
    res->key = q.model_key;
    res->hash = r->hash;
    res->n = n;
    res->m = m;
    res->p = p;
    res->block = mblock;
    res->bytes = nd.model;
    reduced_layout(mblock, n, m, p, &res->rm);
    c->residents.push_back(std::move(up));
    c->stats.reductions++;
  } else {
    c->stats.reduction_cache_hits++;
  }
  res->refs++;
  res->last_use = ++c->use_clock;
  r->model = res;
  r->reused = !needs_model;
  // what the request's sweeps have to wait for
  if (needs_model) res->ready = pass_ref(c->pass);
  if (needs_model || q.mem == LTI_MEM_HOST) r->ready = pass_ref(c->pass);
  if (!needs_model) r->model_ready = pass_ref(res->ready);
  r->block = block;
  r->block_bytes = nd.block();

  char* b = static_cast<char*>(block);
  HostStage& hs = r->hs;
  const bool host = q.mem == LTI_MEM_HOST;
  const double* d_omega = q.omega;
  double* d_G = q.G_out;
  lti_point_info* d_info = q.info_out;
  hipError_t e = hipSuccess;
  ReduceJob job{};
  if (needs_model) {
    job.A = q.A;
    job.B = q.B;
    job.C = q.C;
    job.D = q.D;
  }
  if (host) {
    // A..D (when this request reduces its model) and omega sit back to back
    // in staging; the block mirrors that layout, so one H2D copy moves them
    const size_t src0 = needs_model ? hs.offA : hs.offW;
    const size_t bytes = hs.offW - src0 + sizeof(double) * q.n_omega;
    e = hipMemcpyAsync(b, hs.base + src0, bytes, hipMemcpyHostToDevice, c->rstream);
    jl.copies = true;
    if (needs_model) {
      job.A = reinterpret_cast<const double*>(b);
      job.B = reinterpret_cast<const double*>(b + (hs.offB - hs.offA));
      job.C = reinterpret_cast<const double*>(b + (hs.offC - hs.offA));
      job.D = reinterpret_cast<const double*>(b + (hs.offD - hs.offA));
    }
    b += nd.inputs;
    d_omega = reinterpret_cast<const double*>(b);
    b += nd.omega;
    r->dOffG = (size_t)(b - static_cast<char*>(block));
    d_G = reinterpret_cast<double*>(b);
    b += nd.G;
    d_info = nd.info ? reinterpret_cast<lti_point_info*>(b) : nullptr;
    b += nd.info;
  }
  if (needs_model) {
    job.out = res->rm;
    job.work = nd.work ? reinterpret_cast<double*>(b) : nullptr;
    b += nd.work;
    jl.jobs[reduce_class(n, m, p)].push_back(job);
  }
  ReqDesc& desc = r->desc;
  desc = ReqDesc{};
  desc.H = res->rm.H;
  desc.Bt = res->rm.Bt;
  desc.Ct = res->rm.Ct;
  desc.D = res->rm.D;
  desc.H32 = res->rm.H32;
  desc.Bt32 = res->rm.Bt32;
  desc.Ct32 = res->rm.Ct32;
  desc.omega = d_omega;
  desc.G = d_G;
  desc.info = d_info;
  desc.n = n;
  desc.m = m;
  desc.p = p;
  desc.precision = q.precision;
  desc.rtol = q.rtol;
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return true;
  }
  r->K = q.n_omega;
  // Kernel family: four frequencies per wavefront (n <= 64, at most four
  // right-hand-side columns per tile), one frequency per wavefront
  // (n <= 256), or one frequency per workgroup (n <= 1024, float64; refined
  // requests of that size run the float64 path and report it per point).
  const bool wg = n > kMaxN;
  const bool four = !wg && c->use_sweep16 && sweep16_class(q.precision, n, std::min(m, 4)) >= 0;
  int F = c->tile_points;
  if (F <= 0) F = four ? 4 : wg ? 1 : (int)std::min<int64_t>(8, std::max<int64_t>(1, r->K / 2048));
  if (four) F = (F + 3) & ~3;
  r->F = F;
  // Split the right-hand-side columns over several tiles (each split
  // repeats the rotations) only while the device would otherwise be short of
  // wavefronts: the target counts the waves of tiles already outstanding.
  const int64_t fblocks = (r->K + F - 1) / F;
  const int64_t target = four ? c->target_tiles16 : c->target_tiles;
  const int64_t avail = std::max<int64_t>(0, target - c->outstanding_waves);
  int S = c->rhs_split;
  if (S <= 0) S = (fblocks >= avail) ? 1 : (int)((avail + fblocks - 1) / fblocks);
  S = std::max(1, std::min(S, m));
  if (four || wg) S = std::max(S, (m + 3) / 4);
  r->mc = (m + S - 1) / S;
  r->S = (m + r->mc - 1) / r->mc;
  if (wg)
    r->kclass = kNumSweepClasses + kNumSweep16Classes + sweep_wg_class(LTI_PREC_FP64, n, r->mc);
  else if (four)
    r->kclass = kNumSweepClasses + sweep16_class(q.precision, n, r->mc);
  else {
    // one-frequency kernels keep R * MM <= 32 (R = 1, 2, 4 row slices):
    // split further until the column count fits
    while (sweep_class(q.precision, n, r->mc) < 0 && r->mc > 1) {
      ++S;
      r->mc = (m + S - 1) / S;
      r->S = (m + r->mc - 1) / r->mc;
    }
    r->kclass = sweep_class(q.precision, n, r->mc);
  }
  r->stage = (four || wg) ? 0 : stage_bytes(q.precision, n, m, p);
  r->ntiles = fblocks * r->S;
  r->waves_per_tile = wg ? 4 : 1;
  c->outstanding_waves += r->ntiles * r->waves_per_tile;
  r->next_tile = 0;
  r->tiles_done = 0;
  r->state = RState::kLive;
  r->res.t_admit_us = c->now_us();
  r->res.reduction_reused = r->reused ? 1 : 0;
  return true;
}

void admit(lti_ctx* c) {
  if (c->pending.empty()) return;
  // an idle admission stream, or wait for one (requests that arrive
  // meanwhile join the next pass; queueing a pass behind a running one split
  // the passes and measured slower)
  int rs = -1;
  for (int i = 0; i < c->n_rstreams && rs < 0; ++i) {
    const int cand = (c->next_rstream + i) % c->n_rstreams;
    PassEvent*& lp = c->last_pass[cand];
    if (!lp || hipEventQuery(lp->ev) != hipErrorNotReady) {
      pass_release(c, lp);
      rs = cand;
    }
  }
  if (rs < 0) return;
  JobLists jl;
  // with no sweeps outstanding the pass goes on the stream the next sweep
  // batch will use, which orders the two without a cross-stream wait
  c->rstream = c->inflight.empty() ? c->sstreams[c->next_sstream] : c->rstreams[rs];
  PassEvent* pe = new PassEvent{};
  pe->stream = c->rstream;
  pe->ev = get_event(c, false);
  pe->refs = 1;  // this pass's own reference, dropped below
  c->pass_events.push_back(pe);
  c->pass = pe;
  struct Drop {
    lti_ctx* c;
    PassEvent* pe;
    ~Drop() {
      c->pass = nullptr;
      pass_release(c, pe);
    }
  } drop{c, pe};
  while (!c->pending.empty() && !c->device_error) {
    Request* r = c->pending.front();
    if (!admit_one(c, r, jl)) break;
    c->pending.pop_front();
    if (r->state == RState::kLive) c->live.push_back(r);
  }
  if (c->device_error || (jl.total() == 0 && !jl.copies)) return;
  c->next_rstream = (rs + 1) % c->n_rstreams;
  const bool timed = (c->flags & LTI_CFG_KERNEL_TIMING) != 0 && jl.total() > 0;
  TimedPair tp{nullptr, nullptr};
  hipError_t e = hipSuccess;
  if (timed) {
    tp.a = get_event(c, true);
    tp.b = get_event(c, true);
    e = hipEventRecord(tp.a, c->rstream);
  }
  // the jobs travel in the kernel arguments, kMaxInlineJobs per launch
  ReduceLaunch L;
  for (int rc = 0; rc < kNumReduceClasses && e == hipSuccess; ++rc) {
    const std::vector<ReduceJob>& v = jl.jobs[rc];
    for (size_t i0 = 0; i0 < v.size() && e == hipSuccess; i0 += kMaxInlineJobs) {
      L.njobs = (int)std::min<size_t>(kMaxInlineJobs, v.size() - i0);
      std::copy(v.begin() + i0, v.begin() + i0 + L.njobs, L.job);
      e = launch_reduce(L, rc, c->rstream);
    }
  }
  if (timed && e == hipSuccess) {
    e = hipEventRecord(tp.b, c->rstream);
    c->reduce_timing.push_back(tp);
  }
  // the sweeps of this pass's requests wait on this
  if (e == hipSuccess) e = (pe->ev ? hipEventRecord(pe->ev, c->rstream) : hipErrorOutOfMemory);
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return;
  }
  c->last_pass[rs] = pass_ref(pe);
}

// Gather up to batch_tiles tiles from the live requests (oldest first) into
// one batch: one launch per kernel class and kMaxSegs requests, each request
// a contiguous range of its tiles.
void launch(lti_ctx* c) {
  if (c->live.empty() || (int)c->inflight.size() >= c->max_inflight) return;
  constexpr int kAllClasses = kNumSweepClasses + kNumSweep16Classes + kNumSweepWGClasses;
  struct Piece {
    Request* r;
    int64_t first, count;
  };
  std::vector<std::vector<Piece>> per(kAllClasses);
  std::vector<size_t> lds(kAllClasses, 0);
  Batch b;
  int64_t total = 0;
  // Requests whose uploads and reductions have finished go first.  When none
  // has, the batch takes the requests of the oldest unfinished admission
  // pass only (its launch then waits for that pass on the device), so that a
  // pass admitted later does not hold back the sweeps of an earlier one.
  std::vector<std::pair<const PassEvent*, bool>> seen;
  auto pass_done = [&](const PassEvent* pe) {
    if (!pe || !pe->ev) return true;
    for (const auto& sd : seen)
      if (sd.first == pe) return sd.second;
    // an event in error counts as not done: the launch then waits on it and
    // the wait reports the error
    const bool done = hipEventQuery(pe->ev) == hipSuccess;
    seen.emplace_back(pe, done);
    return done;
  };
  bool any_ready = false;
  const PassEvent* oldest = nullptr;
  for (Request* r : c->live) {
    if (r->state != RState::kLive || r->next_tile >= r->ntiles) continue;
    const bool rd = pass_done(r->ready), md = pass_done(r->model_ready);
    if (rd && md) {
      any_ready = true;
      break;
    }
    if (!oldest) oldest = rd ? r->model_ready : r->ready;
  }
  auto eligible = [&](const Request* r) {
    const bool rd = pass_done(r->ready), md = pass_done(r->model_ready);
    if (any_ready) return rd && md;
    return (rd || r->ready == oldest) && (md || r->model_ready == oldest);
  };
  for (Request* r : c->live) {
    if (total >= c->batch_tiles) break;
    if (r->state != RState::kLive || r->next_tile >= r->ntiles) continue;
    if (!eligible(r)) continue;
    const int64_t take = std::min<int64_t>(r->ntiles - r->next_tile, c->batch_tiles - total);
    per[r->kclass].push_back(Piece{r, r->next_tile, take});
    lds[r->kclass] = std::max(lds[r->kclass], r->stage);
    r->next_tile += take;
    total += take;
    b.credit.emplace_back(r, take);
    if (r->res.t_first_launch_us == 0.0) r->res.t_first_launch_us = c->now_us();
  }
  if (total == 0) return;
  hipError_t e = hipSuccess;
  hipStream_t ss = c->sstreams[c->next_sstream];
  c->next_sstream = (c->next_sstream + 1) % c->n_sstreams;
  b.stream = ss;
  // wait for the uploads and reductions the batch's requests depend on
  std::vector<PassEvent*> waited;
  for (auto& cr : b.credit)
    for (PassEvent* pe : {cr.first->ready, cr.first->model_ready})
      if (pe && pe->stream != ss && !pass_done(pe) && std::find(waited.begin(), waited.end(), pe) == waited.end()) {
        waited.push_back(pe);
        if (e == hipSuccess) e = hipStreamWaitEvent(ss, pe->ev, 0);
      }
  b.timed = (c->flags & LTI_CFG_KERNEL_TIMING) != 0;
  if (b.timed) {
    b.t0 = get_event(c, true);
    b.t1 = get_event(c, true);
    if (e == hipSuccess) e = hipEventRecord(b.t0, ss);
  }
  SweepLaunch L;
  for (int k = 0; k < kAllClasses && e == hipSuccess; ++k) {
    const std::vector<Piece>& v = per[k];
    for (size_t i0 = 0; i0 < v.size() && e == hipSuccess; i0 += kMaxSegs) {
      L.nseg = (int)std::min<size_t>(kMaxSegs, v.size() - i0);
      uint32_t t = 0;
      for (int sgi = 0; sgi < L.nseg; ++sgi) {
        const Piece& pc = v[i0 + sgi];
        SweepSeg& sg = L.seg[sgi];
        sg.rd = pc.r->desc;
        sg.tile0 = t;
        sg.first = (uint32_t)pc.first;
        sg.K = (uint32_t)pc.r->K;
        sg.F = (uint16_t)pc.r->F;
        sg.S = (uint8_t)pc.r->S;
        sg.mc = (uint8_t)pc.r->mc;
        t += (uint32_t)pc.count;
      }
      L.ntiles = (int)t;
      if (k >= kNumSweepClasses + kNumSweep16Classes)
        e = launch_sweep_wg(k - kNumSweepClasses - kNumSweep16Classes, L, ss);
      else if (k >= kNumSweepClasses)
        e = launch_sweep16(k - kNumSweepClasses, L, ss);
      else
        e = launch_sweep(k, L, c->stage_lds ? lds[k] : 0, ss);
      c->stats.sweep_launches++;
    }
  }
  if (b.timed && e == hipSuccess) e = hipEventRecord(b.t1, ss);
  b.done = get_event(c, false);
  if (e == hipSuccess) e = hipEventRecord(b.done, ss);
  c->stats.tiles_launched += total;
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return;
  }
  c->inflight.push_back(std::move(b));
}

void complete_request(lti_ctx* c, Request* r) {
  const lti_request& q = r->req;
  r->res.status = LTI_OK;
  r->res.n_points = q.n_omega;
  if (q.mem == LTI_MEM_HOST) {
    HostStage& hs = r->hs;
    std::memcpy(q.G_out, hs.base + hs.offG, sizeof(double) * 2 * (size_t)q.n_omega * q.ny * q.nu);
    if (q.info_out) {
      std::memcpy(q.info_out, hs.base + hs.offInfo, sizeof(lti_point_info) * q.n_omega);
      for (int64_t k = 0; k < q.n_omega; ++k) {
        const lti_point_info& pi = q.info_out[k];
        if (pi.path == LTI_PATH_REFINED) r->res.n_refined++;
        if (pi.path == LTI_PATH_FALLBACK) r->res.n_fallback++;
        if (pi.path == LTI_PATH_SINGULAR) r->res.n_singular++;
        r->res.max_est_rel_err = std::max(r->res.max_est_rel_err, (double)pi.est_rel_err);
      }
    }
  }
  release_stage(c, r->hs);
  r->res.t_done_us = c->now_us();
  r->state = RState::kDone;
  c->stats.requests_done++;
  c->stats.points_done += q.n_omega;
  release_request_memory(c, r);
}

void finish_tiles(lti_ctx* c, Request* r) {
  const lti_request& q = r->req;
  if (q.mem == LTI_MEM_DEVICE) {
    // results are already in the caller's device buffers; the batch event
    // that credited the last tile orders them
    complete_request(c, r);
    return;
  }
  HostStage& hs = r->hs;
  char* b = static_cast<char*>(r->block);
  // G and info are back to back in the block and in staging (same aligned
  // offsets): one D2H copy
  const size_t gbytes = sizeof(double) * 2 * (size_t)q.n_omega * q.ny * q.nu;
  const size_t bytes = q.info_out ? (hs.offInfo - hs.offG) + sizeof(lti_point_info) * q.n_omega : gbytes;
  hipError_t e = hipMemcpyAsync(hs.base + hs.offG, b + r->dOffG, bytes, hipMemcpyDeviceToHost, c->stream);
  r->d2h_ev = get_event(c, false);
  if (e == hipSuccess) e = hipEventRecord(r->d2h_ev, c->stream);
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return;
  }
  r->state = RState::kFinishing;
}

bool retire(lti_ctx* c) {
  bool progressed = false;
  while (!c->reduce_timing.empty()) {
    TimedPair& tp = c->reduce_timing.front();
    const hipError_t q = hipEventQuery(tp.b);
    if (q == hipErrorNotReady) break;
    float ms = 0.f;
    if (q == hipSuccess && hipEventElapsedTime(&ms, tp.a, tp.b) == hipSuccess) {
      c->stats.reduce_kernel_ms += ms;
      c->stats.timed_reduce_launches++;
    }
    put_event(c, tp.a, true);
    put_event(c, tp.b, true);
    c->reduce_timing.pop_front();
  }
  // batches on different sweep streams may finish in any order
  for (auto bit = c->inflight.begin(); bit != c->inflight.end();) {
    Batch& b = *bit;
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) {
      ++bit;
      continue;
    }
    if (q != hipSuccess) {
      fail_all(c, LTI_EDEVICE);
      return true;
    }
    if (b.timed) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, b.t0, b.t1) == hipSuccess) {
        c->stats.sweep_kernel_ms += ms;
        c->stats.timed_sweep_launches++;
      }
      put_event(c, b.t0, true);
      put_event(c, b.t1, true);
    }
    for (auto& cr : b.credit) {
      Request* r = cr.first;
      r->tiles_done += cr.second;
      c->outstanding_waves -= cr.second * r->waves_per_tile;
      if (r->tiles_done == r->ntiles && r->state == RState::kLive) finish_tiles(c, r);
      if (c->device_error) return true;
    }
    put_event(c, b.done, false);
    bit = c->inflight.erase(bit);
    progressed = true;
  }
  for (auto it = c->live.begin(); it != c->live.end();) {
    Request* r = *it;
    if (r->state == RState::kFinishing) {
      const hipError_t q = hipEventQuery(r->d2h_ev);
      if (q == hipErrorNotReady) {
        ++it;
        continue;
      }
      put_event(c, r->d2h_ev, false);
      r->d2h_ev = nullptr;
      if (q != hipSuccess) {
        fail_all(c, LTI_EDEVICE);
        return true;
      }
      complete_request(c, r);
    }
    if (r->state == RState::kDone || r->state == RState::kFailed) {
      it = c->live.erase(it);
      progressed = true;
      c->cv_done.notify_all();
    } else {
      ++it;
    }
  }
  return progressed;
}

// One scheduling pass (c->mu held, c->device current): retire finished work,
// admit pending requests, launch tiles.  Returns whether anything changed.
bool pump(lti_ctx* c) {
  if (c->device_error) return false;
  bool progressed = retire(c);
  const size_t inflight_before = c->inflight.size();
  auto fill = [&] {
    while ((int)c->inflight.size() < c->max_inflight && !c->device_error) {
      const size_t sz = c->inflight.size();
      launch(c);
      if (c->inflight.size() == sz) break;
    }
  };
  // sweeps of requests already admitted go out before a new admission pass,
  // so that the pass does not land on an idle sweep stream ahead of them
  fill();
  const size_t pending_before = c->pending.size();
  admit(c);
  progressed |= c->pending.size() != pending_before;
  fill();
  progressed |= c->inflight.size() != inflight_before;
  return progressed;
}

void destroy_admit_streams(lti_ctx* c) {
  for (int i = 0; i < kAdmitStreams; ++i) {
    if (c->rstreams[i]) (void)hipStreamDestroy(c->rstreams[i]);
    c->rstreams[i] = nullptr;
  }
  for (int i = 1; i < kSweepStreams; ++i) {  // [0] is c->stream
    if (c->sstreams[i]) (void)hipStreamDestroy(c->sstreams[i]);
    c->sstreams[i] = nullptr;
  }
}

bool busy(const lti_ctx* c) {
  return !c->inflight.empty() || !c->live.empty() || !c->reduce_timing.empty() || !c->pending.empty();
}

// Makes the context's device current on the calling thread for a scope and
// restores the caller's device afterwards.
struct DeviceScope {
  int prev = -1;
  explicit DeviceScope(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  DeviceScope(const DeviceScope&) = delete;
  DeviceScope& operator=(const DeviceScope&) = delete;
  ~DeviceScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void scheduler(lti_ctx* c) {
  (void)hipSetDevice(c->device);
  // short sleeps below must stay short: 1 us timer slack for this thread
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0, 0, 0);
  std::unique_lock<std::mutex> lk(c->mu);
  Clock::time_point idle_since = Clock::now();
  while (!c->stop) {
    if (c->device_error) {
      c->cv_work.wait(lk, [&] { return c->stop; });
      break;
    }
    if (pump(c)) {
      idle_since = Clock::now();
      continue;
    }
    if (busy(c)) {
      // device work outstanding: poll its events, spinning (yield) for the
      // first 200 us so that short requests complete without sleep latency;
      // while a caller's thread runs the passes itself (submit, poll), step
      // back so as not to contend with it for the lock
      lk.unlock();
      if (c->now_us() - c->client_pump_us.load(std::memory_order_relaxed) < kClientActiveUs)
        std::this_thread::sleep_for(std::chrono::microseconds(20));
      else if (Clock::now() - idle_since < std::chrono::microseconds(200))
        std::this_thread::yield();
      else
        std::this_thread::sleep_for(std::chrono::microseconds(10));
      lk.lock();
    } else {
      c->cv_work.wait_for(lk, std::chrono::milliseconds(5));
      idle_since = Clock::now();
    }
  }
}

int validate(const lti_request* q) {
  if (!q) return LTI_EINVAL;
  if (q->nx <= 0 || q->nu <= 0 || q->ny <= 0 || q->n_omega <= 0) return LTI_EINVAL;
  if (!q->A || !q->B || !q->C || !q->omega || !q->G_out) return LTI_EINVAL;
  if (q->mem != LTI_MEM_HOST && q->mem != LTI_MEM_DEVICE) return LTI_EINVAL;
  if (q->precision != LTI_PREC_FP64 && q->precision != LTI_PREC_REFINED) return LTI_EINVAL;
  if (q->reserved0 != 0) return LTI_EINVAL;
  if (q->n_omega > (int64_t)UINT32_MAX) return LTI_EINVAL;
  if (std::isnan(q->rtol) || q->rtol >= 1.0) return LTI_EINVAL;
  if (q->nx > kMaxNWG || q->nu > kMaxRhs || q->ny > kMaxRhs) return LTI_EUNSUPPORTED;
  // tile indices (at most n_omega x nu per request) are 32-bit
  if (q->n_omega * q->nu > (int64_t)UINT32_MAX) return LTI_EUNSUPPORTED;
  return LTI_OK;
}

// Stage a host-memory request's inputs (and room for its outputs).
int stage_inputs(lti_ctx* c, Request* r) {
  const lti_request& q = r->req;
  const int n = q.nx, m = q.nu, p = q.ny;
  HostStage& hs = r->hs;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align_up(bytes);
    return o;
  };
  hs.offA = take(sizeof(double) * n * n);
  hs.offB = take(sizeof(double) * n * m);
  hs.offC = take(sizeof(double) * p * n);
  hs.offD = take(sizeof(double) * p * m);
  hs.offW = take(sizeof(double) * q.n_omega);
  hs.offG = take(sizeof(double) * 2 * (size_t)q.n_omega * p * m);
  hs.offInfo = take(q.info_out ? sizeof(lti_point_info) * q.n_omega : 0);
  hs.bytes = off;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    hs.base = static_cast<char*>(c->staging.alloc(hs.bytes));
  }
  hs.pinned = hs.base != nullptr;
  if (!hs.pinned) {
    try {
      hs.fallback.resize(hs.bytes);
    } catch (...) {
      return LTI_ENOMEM;
    }
    hs.base = hs.fallback.data();
  }
  // A..D must be contiguous in this order (one H2D copy)
  std::memcpy(hs.base + hs.offA, q.A, sizeof(double) * n * n);
  std::memcpy(hs.base + hs.offB, q.B, sizeof(double) * n * m);
  std::memcpy(hs.base + hs.offC, q.C, sizeof(double) * p * n);
  if (q.D)
    std::memcpy(hs.base + hs.offD, q.D, sizeof(double) * p * m);
  else
    std::memset(hs.base + hs.offD, 0, sizeof(double) * p * m);
  std::memcpy(hs.base + hs.offW, q.omega, sizeof(double) * q.n_omega);
  // the model's identity: its dimensions and the bytes of A, B, C, D (not
  // the alignment gaps between them in staging, which hold whatever the
  // pool held before); only keyed requests are ever matched
  r->hash = 0;
  if (q.model_key == 0) return LTI_OK;
  uint64_t h = 1469598103934665603ull;
  const int dims[3] = {n, m, p};
  h = fnv1a(dims, sizeof(dims), h);
  h = fnv1a(hs.base + hs.offA, sizeof(double) * n * n, h);
  h = fnv1a(hs.base + hs.offB, sizeof(double) * n * m, h);
  h = fnv1a(hs.base + hs.offC, sizeof(double) * p * n, h);
  h = fnv1a(hs.base + hs.offD, sizeof(double) * p * m, h);
  r->hash = h;
  return LTI_OK;
}

}  // namespace

extern "C" {

uint32_t lti_freqresp_abi_version(void) { return LTI_ABI_VERSION; }

const char* lti_freqresp_strerror(int code) {
  switch (code) {
    case LTI_OK: return "ok";
    case LTI_PENDING: return "request still pending";
    case LTI_EINVAL: return "invalid argument";
    case LTI_ENOSPC: return "request can never fit in the arena";
    case LTI_EAGAIN: return "pending queue full";
    case LTI_ENOENT: return "unknown or already collected request";
    case LTI_EDEVICE: return "HIP device error; context unusable";
    case LTI_ENOMEM: return "host allocation failed";
    case LTI_EUNSUPPORTED: return "dimensions not supported by the kernels";
    default: return "unknown error code";
  }
}

int lti_freqresp_create(const lti_config* cfg, lti_ctx** out) {
  if (!cfg || !out) return LTI_EINVAL;
  *out = nullptr;
  if (cfg->abi_version != LTI_ABI_VERSION) return LTI_EINVAL;
  if (!cfg->arena || cfg->arena_bytes < (size_t(1) << 20)) return LTI_EINVAL;
  if (reinterpret_cast<uintptr_t>(cfg->arena) % kAlign) return LTI_EINVAL;
  std::unique_ptr<lti_ctx> c(new (std::nothrow) lti_ctx());
  if (!c) return LTI_ENOMEM;
  c->device = cfg->device;
  c->flags = cfg->flags;
  c->max_pending = cfg->max_pending > 0 ? cfg->max_pending : kDefaultMaxPending;
  c->tile_points = cfg->tile_points > 0 ? cfg->tile_points : 0;
  c->batch_tiles = cfg->max_batch_tiles > 0 ? cfg->max_batch_tiles : kDefaultBatchTiles;
  // debug knobs for tuning sweeps (not part of the ABI)
  if (const char* e = std::getenv("LTI_FREQRESP_RHS_SPLIT")) c->rhs_split = std::atoi(e);
  if (const char* e = std::getenv("LTI_FREQRESP_TARGET_TILES")) c->target_tiles = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_STAGE_LDS")) c->stage_lds = std::atoi(e) != 0;
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP16")) c->use_sweep16 = std::atoi(e) != 0;
  if (const char* e = std::getenv("LTI_FREQRESP_TARGET_TILES16")) c->target_tiles16 = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_MAX_INFLIGHT"))
    c->max_inflight = std::max(1, std::min(64, std::atoi(e)));
  if (const char* e = std::getenv("LTI_FREQRESP_ADMIT_STREAMS"))
    c->n_rstreams = std::max(1, std::min(kAdmitStreams, std::atoi(e)));
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP_STREAMS"))
    c->n_sstreams = std::max(1, std::min(kSweepStreams, std::atoi(e)));
  c->t0 = Clock::now();
  if (hipSetDevice(c->device) != hipSuccess) return LTI_EDEVICE;
  c->arena.init(static_cast<char*>(cfg->arena), cfg->arena_bytes);
  const size_t staging = cfg->host_staging_bytes ? cfg->host_staging_bytes : kDefaultStaging;
  void* hp = nullptr;
  if (hipHostMalloc(&hp, staging, hipHostMallocDefault) != hipSuccess) return LTI_EDEVICE;
  c->staging_block = static_cast<char*>(hp);
  c->staging.init(c->staging_block, staging);
  // tuning knob (not part of the ABI): keep the sweeps off the first N CUs,
  // so that reductions always find room beside them
  int reserved_cus = 0;
  if (const char* e = std::getenv("LTI_FREQRESP_RESERVED_CUS")) reserved_cus = std::max(0, std::atoi(e));
  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
  } else {
    hipError_t e = hipSuccess;
    int ncu = 0;
    if (reserved_cus > 0 &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        reserved_cus < ncu) {
      std::vector<uint32_t> mask((ncu + 31) / 32, 0u);
      for (int cu = reserved_cus; cu < ncu; ++cu) mask[cu / 32] |= 1u << (cu % 32);
      e = hipExtStreamCreateWithCUMask(&c->stream, (uint32_t)mask.size(), mask.data());
    } else {
      e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    }
    if (e != hipSuccess) {
      (void)hipHostFree(hp);
      return LTI_EDEVICE;
    }
    c->own_stream = true;
  }
  bool ok = true;
  for (int i = 0; i < c->n_rstreams && ok; ++i)
    ok = hipStreamCreateWithFlags(&c->rstreams[i], hipStreamNonBlocking) == hipSuccess;
  c->sstreams[0] = c->stream;
  for (int i = 1; i < c->n_sstreams && ok; ++i)
    ok = hipStreamCreateWithFlags(&c->sstreams[i], hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    destroy_admit_streams(c.get());
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    (void)hipHostFree(hp);
    return LTI_EDEVICE;
  }
  try {
    c->thread = std::thread(scheduler, c.get());
  } catch (...) {
    (void)hipHostFree(hp);
    destroy_admit_streams(c.get());
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    return LTI_ENOMEM;
  }
  *out = c.release();
  return LTI_OK;
}

int lti_freqresp_submit(lti_ctx* c, const lti_request* q, uint64_t* out_id) {
  if (!c || !out_id) return LTI_EINVAL;
  const int v = validate(q);
  if (v != LTI_OK) return v;
  const int n = q->nx, m = q->nu, p = q->ny;
  if (q->mem == LTI_MEM_HOST) {
    if (!all_finite(q->A, (size_t)n * n) || !all_finite(q->B, (size_t)n * m) || !all_finite(q->C, (size_t)p * n) ||
        (q->D && !all_finite(q->D, (size_t)p * m)) || !all_finite(q->omega, (size_t)q->n_omega))
      return LTI_EINVAL;
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return LTI_ENOMEM;
  r->req = *q;
  if (q->rtol <= 0.0) r->req.rtol = 1e-10;
  if (q->mem == LTI_MEM_HOST) {
    // checked before staging (the pinned pool is not taken for a request
    // that can never run); device requests check under the lock below
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->device_error) return LTI_EDEVICE;
    const Need nd = request_need(r->req, true);
    if (!c->arena.can_ever_fit(nd.block() + nd.model)) return LTI_ENOSPC;
    if ((int)c->all.size() >= c->max_pending) return LTI_EAGAIN;
  }
  if (q->mem == LTI_MEM_HOST) {
    const int s = stage_inputs(c, r.get());
    if (s != LTI_OK) return s;
  } else {
    r->hash = 0;  // device inputs: the key and dimensions identify the model
  }
  std::lock_guard<std::mutex> lk(c->mu);
  if (c->device_error) {
    release_stage(c, r->hs);
    return LTI_EDEVICE;
  }
  if (q->mem == LTI_MEM_DEVICE) {
    const Need nd = request_need(r->req, true);
    if (!c->arena.can_ever_fit(nd.block() + nd.model)) return LTI_ENOSPC;
  }
  if ((int)c->all.size() >= c->max_pending) {
    release_stage(c, r->hs);
    return LTI_EAGAIN;
  }
  r->id = c->next_id++;
  r->res.t_submit_us = c->now_us();
  Request* raw = r.get();
  c->all.emplace(raw->id, std::move(r));
  c->pending.push_back(raw);
  c->stats.requests_submitted++;
  *out_id = raw->id;
  {
    // start it from this thread when it can start now
    DeviceScope ds(c->device);
    pump(c);
    c->client_pump_us.store(c->now_us(), std::memory_order_relaxed);
  }
  c->cv_work.notify_one();
  return LTI_OK;
}

int lti_freqresp_poll(lti_ctx* c, uint64_t id, int32_t timeout_us, lti_result* out) {
  if (!c) return LTI_EINVAL;
  std::unique_lock<std::mutex> lk(c->mu);
  auto it = c->all.find(id);
  if (it == c->all.end()) return LTI_ENOENT;
  Request* r = it->second.get();
  auto finished = [&] { return r->state == RState::kDone || r->state == RState::kFailed; };
  if (!finished() && timeout_us != 0) {
    // drive the scheduling passes from this thread for a while (a short
    // request completes without a thread hand-off), then sleep on the
    // completion signal
    const Clock::time_point t_start = Clock::now();
    const auto limit = std::chrono::microseconds(
        timeout_us < 0 ? kPollSpinUs : std::min<int64_t>(timeout_us, kPollSpinUs));
    {
      DeviceScope ds(c->device);
      while (!finished() && !c->device_error && Clock::now() - t_start < limit) {
        const bool progressed = pump(c);
        c->client_pump_us.store(c->now_us(), std::memory_order_relaxed);
        if (progressed) continue;
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      }
    }
    if (!finished()) {
      if (timeout_us < 0) {
        c->cv_done.wait(lk, finished);
      } else {
        const auto left = std::chrono::microseconds(timeout_us) - (Clock::now() - t_start);
        if (left > Clock::duration::zero()) c->cv_done.wait_for(lk, left, finished);
      }
    }
  }
  if (!finished()) return LTI_PENDING;
  const int status = r->state == RState::kDone ? LTI_OK : r->status;
  r->res.status = status;
  if (out) *out = r->res;
  release_stage(c, r->hs);
  c->all.erase(it);
  return status;
}

int lti_freqresp_destroy(lti_ctx* c) {
  if (!c) return LTI_EINVAL;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    c->stop = true;
  }
  c->cv_work.notify_all();
  c->cv_done.notify_all();
  if (c->thread.joinable()) c->thread.join();
  (void)hipSetDevice(c->device);
  for (hipStream_t rs : c->rstreams)
    if (rs) (void)hipStreamSynchronize(rs);
  for (hipStream_t ss : c->sstreams)
    if (ss) (void)hipStreamSynchronize(ss);
  for (auto& b : c->inflight) {
    put_event(c, b.done, false);
    put_event(c, b.t0, true);
    put_event(c, b.t1, true);
  }
  for (auto& tp : c->reduce_timing) {
    put_event(c, tp.a, true);
    put_event(c, tp.b, true);
  }
  for (auto& kv : c->all)
    if (kv.second->d2h_ev) put_event(c, kv.second->d2h_ev, false);
  for (PassEvent*& lp : c->last_pass) lp = nullptr;
  for (PassEvent* pe : c->pass_events) {
    put_event(c, pe->ev, false);
    delete pe;
  }
  c->pass_events.clear();
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->timing_pool) (void)hipEventDestroy(e);
  if (c->staging_block) (void)hipHostFree(c->staging_block);
  destroy_admit_streams(c);
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return LTI_OK;
}

int lti_freqresp_get_reduced(lti_ctx* c, uint64_t key, int32_t nx, int32_t nu, int32_t ny, double* H, double* Bt,
                             double* Ct) {
  if (!c || key == 0 || nx <= 0 || nu <= 0 || ny <= 0) return LTI_EINVAL;
  ReducedModel rm{};
  Resident* held = nullptr;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->device_error) return LTI_EDEVICE;
    for (auto& up : c->residents)
      if (up->key == key && up->n == nx && up->m == nu && up->p == ny) held = up.get();
    if (!held) return LTI_ENOENT;
    rm = held->rm;
    held->refs++;
  }
  const int n = nx, m = nu, p = ny;
  std::vector<double> hp((size_t)hlen(n)), bt((size_t)n * m), ct((size_t)n * p);
  hipError_t e = hipSetDevice(c->device);
  for (hipStream_t rs : c->rstreams)
    if (e == hipSuccess) e = hipStreamSynchronize(rs);
  for (hipStream_t ss : c->sstreams)
    if (e == hipSuccess) e = hipStreamSynchronize(ss);
  if (e == hipSuccess) e = hipMemcpy(hp.data(), rm.H, hp.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(bt.data(), rm.Bt, bt.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(ct.data(), rm.Ct, ct.size() * 8, hipMemcpyDeviceToHost);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    held->refs--;
  }
  if (e != hipSuccess) return LTI_EDEVICE;
  if (H) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) H[(size_t)i * n + j] = (i <= j + 1) ? hp[hoff(j) + i] : 0.0;
  }
  if (Bt) std::memcpy(Bt, bt.data(), bt.size() * 8);
  if (Ct) {
    for (int a = 0; a < p; ++a)
      for (int i = 0; i < n; ++i) Ct[(size_t)a * n + i] = ct[(size_t)i * p + a];
  }
  return LTI_OK;
}

int lti_freqresp_stats(lti_ctx* c, lti_stats* out) {
  if (!c || !out) return LTI_EINVAL;
  std::lock_guard<std::mutex> lk(c->mu);
  *out = c->stats;
  out->arena_bytes_in_use = c->arena.used();
  out->arena_peak_bytes = c->arena.peak();
  return LTI_OK;
}

}  // extern "C"
