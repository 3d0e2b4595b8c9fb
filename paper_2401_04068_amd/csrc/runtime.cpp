// Serving runtime behind the C ABI: arena sub-allocation, resident reduced
// models, admission by memory budget, and continuous batching of the
// per-frequency solves of every live request into shared kernel launches.
//
// Device work is issued by a scheduling pass (pump) that runs under the
// context lock: on the context's scheduler thread, and inline on the caller's
// thread in submit() and in a waiting poll(), so a lone request starts and
// completes without a thread hand-off.  A pass:
//
//   admit    pending requests in arrival order while their memory fits:
//            upload inputs, clear their refinement queues, reuse a resident
//            reduced model or queue a reduction job (the jobs of one pass go
//            to the device as one table and share a launch per kernel
//            class).  Uploads and reductions go to an idle one of
//            kAdmitStreams admission streams and end with an event that the
//            requests of the pass (and the models it reduced) keep; a sweep
//            launch first waits on the events of its requests, so reductions
//            run beside sweeps.  While every admission stream is still busy,
//            new requests wait, and are then admitted together: their
//            reductions share launches and run side by side (one reduction
//            occupies a single CU);
//   launch   gather up to max_batch_tiles tiles from the live requests
//            (oldest first), group them by kernel class and launch them on
//            the sweep stream; a request whose last tiles are in the batch is
//            finished in it: the extended refinement of its queued points,
//            then the copy of its results to pinned host memory.  One batch
//            is outstanding, so requests that arrive meanwhile join the next;
//   retire   when a batch's event has fired, credit its tiles; a request
//            whose tiles are all done becomes visible to poll().
//
// Host inputs are copied at submit() into pinned staging owned by the
// library, so every H2D and D2H copy is a true asynchronous DMA that never
// stalls the scheduler behind queued kernels.  The descriptors the sweep
// kernels need (per-request descriptors and tile ranges) travel in the kernel
// arguments; reduction jobs travel as one small table per pass.
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
// Sweep batches outstanding: two.  A new batch is formed when one of the two
// completes, so requests admitted meanwhile share it, and the next batch is
// already queued behind the running one (no host gap between batches).  On
// the 4096-request serving mix two outstanding batches of up to 262,144
// tiles measured 22.8 M points/s refined and 40.1 M float64, against 19.3 and
// 32.0 with one batch of 16,384 tiles; the 64-state stream and the open-loop
// latency were unchanged.
constexpr int kInflight = 2;
// Streams: one admission stream and one sweep stream by default (a process
// gets few hardware queues, four by default, and streams that share one run
// in order).  With one admission stream, requests that arrive during a
// reduction are admitted together afterwards, so their reductions and their
// sweeps share launches; a second admission stream (a tuning knob) measured
// slower.  Every sweep goes to the one sweep stream, which orders a
// request's refinement and result copy after all of its tiles.
constexpr int kAdmitStreams = 2;
// Sweep streams: the context's stream plus auxiliary ones.  A batch's sweep
// launches (one per kernel class) are spread over them: the launches of one
// class often cannot fill the GPU for their whole duration (their waves'
// lifetimes differ several-fold, so a launch ends with a long tail), and on
// one stream the next launch would wait for that tail.  The batch's
// refinement and result copies go to a finishing stream that waits for the
// batch's launches on every stream it used; the sweep streams are not joined
// between batches.
constexpr int kMaxSweepStreams = 3;
// Two by default: with the admission and finishing streams that makes four,
// the hardware queues a process gets by default (more streams share queues
// and then run in order).  Serving mix: 49.7 M points/s refined with two,
// 46.3 with three.
constexpr int kDefaultSweepStreams = 2;
// CUs kept free of sweeps (the library's own sweep streams are created with a
// CU mask without them), so that reductions -- a chain of small launches for
// large models -- find room while sweeps fill the rest of the GPU.
constexpr int kReservedCUs = 0;
// Reduction jobs queued by one admission pass (bounds one pass's work).
constexpr int kMaxJobs = 1024;
constexpr int kDefaultMaxPending = 8192;
constexpr int kDefaultBatchTiles = 262144;
constexpr size_t kDefaultStaging = size_t(256) << 20;
// Requests a sweep batch may finish: the summaries of their point records
// are computed on the device into a per-batch table of this many entries
// (one slot per outstanding batch).
constexpr int kMaxFin = 1024;
// A waiting poll() runs scheduling passes itself for up to this long.
constexpr int64_t kPollSpinUs = 2000;
// The scheduler thread backs off while a caller's thread has run a
// scheduling pass within this window.
constexpr double kClientActiveUs = 200.0;

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

// The end of one admission pass on its stream (uploads, queue clearing and
// reductions), shared by the requests admitted in it and by the models it
// reduced.
struct PassEvent {
  hipEvent_t ev = nullptr;
  hipStream_t stream = nullptr;  // where the pass was issued
  int refs = 0;
};

struct Resident {
  PassEvent* ready = nullptr;  // pass that reduced it, until a user completed
  uint64_t key = 0;
  uint64_t hash = 0;
  int n = 0, m = 0, p = 0;     // the request's sizes
  int trans = 0;
  int desc = 0;                // descriptor system (T stored)
  void* block = nullptr;
  size_t bytes = 0;
  ReducedModel rm{};
  int refs = 0;
  uint64_t last_use = 0;
  size_t slot = 0;             // its index in the context's resident list
};

// kCopy: results in pinned staging, the copy to the caller's arrays not yet
// done (it runs outside the context's lock)
enum class RState { kPending, kLive, kCopy, kDone, kFailed };

// Host memory of a request, from the pinned pool when it has room.
struct HostBuf {
  char* base = nullptr;  // pinned block, or fallback.data()
  size_t bytes = 0;
  bool pinned = false;
  std::vector<char> fallback;
};
// Host-side staging of a request: `in` holds A, B, C, D and omega of a
// host-memory request (copied at submit); `out` receives the results as the
// device returns them, G and the point records (the records only, for
// device-memory requests), and is taken at admission.
struct HostStage {
  HostBuf in, out;
  size_t offA = 0, offB = 0, offC = 0, offD = 0, offE = 0, offW = 0;  // in `in`
  size_t offG = 0, offInfo = 0, offDG = 0, outBytes = 0;     // in `out`
};

struct Request {
  uint64_t id = 0;
  lti_request req{};
  RState state = RState::kPending;
  int status = LTI_OK;
  uint64_t hash = 0;
  HostStage hs;
  int trans = 0;          // the transposed system is solved (ny < nu)
  int sm = 0, sp = 0;     // the solved system's inputs and outputs
  Resident* model = nullptr;
  bool reused = false;
  PassEvent* ready = nullptr;        // its own admission pass
  PassEvent* model_ready = nullptr;  // the pass that reduced a reused model
  void* block = nullptr;  // device: A..D, omega, G, info, queue, reduction scratch
  size_t block_bytes = 0;
  size_t dOffG = 0;       // G (host requests; info follows at the staging offset)
  lti_point_info* dinfo = nullptr;  // the point records on the device
  const PointSummary* sum = nullptr;  // their summary (pinned), set by the finishing batch
  ReqDesc desc{};         // handed to the sweep kernels in their arguments
  int kclass = -1;
  int64_t K = 0;
  int F = 1;        // frequencies per tile
  int S = 1;        // right-hand-side column groups per frequency block
  int mc = 1;       // columns per group
  size_t stage = 0; // LDS bytes a sweep workgroup needs to stage the model
  int64_t ntiles = 0, next_tile = 0, tiles_done = 0;
  int waves_per_tile = 1;
  lti_result res{};
};

struct Batch {
  hipEvent_t done = nullptr;
  std::vector<hipEvent_t> joins;   // the end of the batch's sweeps on each stream it used
  bool joins_timed = false;        // joins come from the timing pool
  std::vector<hipEvent_t> tstart;  // timing: the start of its sweeps on each stream it used
  // with kernel timing: tev[0] before the first kernel, tev[i + 1] after the
  // launches of family tfam[i]
  std::vector<hipEvent_t> tev;
  std::vector<int> tfam;
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

TilePlan plan_tiles(int precision, int n, int sm, int sp, int64_t K, int64_t avail_waves4, int64_t avail_waves1,
                    const TileKnobs& kn) {
  TilePlan t{};
  // Kernel family: four frequencies per wavefront (n <= 64, at most four
  // right-hand-side columns per tile), two frequencies per wavefront
  // (64 < n <= 128, at most four columns per tile), one frequency per
  // wavefront (n <= 256), or one frequency per workgroup (n <= 1024).
  const bool wg = n > kMaxN && !kn.descriptor;
  const bool four = !wg && !kn.descriptor && kn.use_sweep16 && sweep16_class(precision, n, std::min(sm, 4)) >= 0;
  const bool two = !wg && !four && !kn.descriptor && kn.use_sweep32 && sm <= kn.sweep32_max_cols &&
                   sweep32_class(precision, n, std::min(sm, 4)) >= 0;
  int F = kn.tile_points;
  if (F <= 0) F = four ? 4 : two ? 2 : wg ? 1 : (int)std::min<int64_t>(8, std::max<int64_t>(1, K / 2048));
  if (four) F = (F + 3) & ~3;
  if (two) F = (F + 1) & ~1;
  t.F = F;
  // Split the right-hand-side columns over several tiles (each split
  // repeats the rotations) only while the device would otherwise be short of
  // wavefronts: `avail` counts the waves it can still take.
  const int64_t fblocks = (K + F - 1) / F;
  const int64_t avail = four ? avail_waves4 : two ? avail_waves1 / 2 : avail_waves1;
  int S = kn.rhs_split;
  if (S <= 0) S = (fblocks >= avail) ? 1 : (int)((avail + fblocks - 1) / fblocks);
  S = std::max(1, std::min(S, sm));
  if (four || two || wg) S = std::max(S, (sm + 3) / 4);
  t.mc = (sm + S - 1) / S;
  t.S = (sm + t.mc - 1) / t.mc;
  if (wg) {
    t.kclass = kNumSweepClasses + kNumSweep16Classes + sweep_wg_class(precision, n, t.mc);
  } else if (four) {
    t.kclass = kNumSweepClasses + sweep16_class(precision, n, t.mc);
  } else if (two) {
    t.kclass = kSweep32Base + sweep32_class(precision, n, t.mc);
  } else {
    // one-frequency kernels keep R * MM <= 32 (R = 1, 2, 4 row slices):
    // split further until the column count fits
    while (sweep_class(precision, n, t.mc) < 0 && t.mc > 1) {
      ++S;
      t.mc = (sm + S - 1) / S;
      t.S = (sm + t.mc - 1) / t.mc;
    }
    t.kclass = sweep_class(precision, n, t.mc);
    if (kn.descriptor) t.kclass = t.kclass < 0 ? -1 : kSweepDescBase + sweep_class(LTI_PREC_FP64, n, t.mc);
  }
  t.stage = (four || two || wg || kn.descriptor) ? 0 : stage_bytes(precision, n, sm, sp);
  t.ntiles = fblocks * t.S;
  t.waves_per_tile = wg ? 4 : 1;
  return t;
}

hipError_t launch_any_sweep(int k, const SweepLaunch& L, size_t lds_bytes, hipStream_t s) {
  if (k >= kSweep32Base) return launch_sweep32(k - kSweep32Base, L, s);
  if (k >= kSweepDescBase) return launch_sweep_desc(k - kSweepDescBase, L, s);
  if (k >= kNumSweepClasses + kNumSweep16Classes) return launch_sweep_wg(k - kNumSweepClasses - kNumSweep16Classes, L, s);
  if (k >= kNumSweepClasses) return launch_sweep16(k - kNumSweepClasses, L, s);
  return launch_sweep(k, L, lds_bytes, s);
}

namespace {

// Doubles a request's omega array holds.
size_t omega_doubles(const lti_request& q) {
  return (q.points == LTI_POINTS_S ? 2 : 1) * (size_t)q.n_omega;
}

}  // namespace
}  // namespace lti

using namespace lti;

struct lti_ctx {
  int device = 0;
  hipStream_t stream = nullptr;              // sweeps (and passes while no batch is out)
  hipStream_t aux[kMaxSweepStreams - 1] = {};  // more sweep streams
  int n_sweep_streams = kDefaultSweepStreams;
  // the refinement, record summaries and result copies of the requests a
  // batch finishes, after the batch's sweeps on every stream it used; the
  // sweep streams go on with the next batch meanwhile
  hipStream_t fstream = nullptr;
  hipEvent_t union_end = nullptr;  // timing: the latest sweep end of the retired batches
  // batches launched and retired (they retire in order), and the last batch
  // that used each sweep stream and the finishing stream (-1: none)
  int64_t batches_retired = 0;
  int64_t last_use[kMaxSweepStreams + 1] = {-1, -1, -1, -1};
  hipStream_t rstreams[kAdmitStreams] = {};  // uploads and reductions
  int next_rstream = 0;
  int n_rstreams = 1;
  int max_inflight = kInflight;  // sweep batches outstanding
  int n_cus = 256;               // the device's compute units
  hipStream_t rstream = nullptr;             // the current pass's stream
  PassEvent* last_pass[kAdmitStreams] = {};  // the last pass on each
  // reduction job tables, one per admission stream (a pass claims the
  // stream's table only when the stream's previous pass has completed)
  ReduceJob* jobtab_host[kAdmitStreams] = {};
  ReduceJob* jobtab_dev[kAdmitStreams] = {};
  int pass_slot = 0;
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
  bool use_sweep32 = true;  // two-frequencies-per-wavefront kernels where they apply
  // Requests of any width go to the two-frequency kernels, in groups of four
  // columns: measured, groups of four with two frequencies per wavefront
  // outrun the one-frequency kernels that hold 8 or 16 columns at once.
  int sweep32_max_cols = kMaxRhs;
  int64_t target_tiles16 = kTargetTilesFour;
  int64_t target_tiles = kTargetTilesOne;
  int64_t outstanding_waves = 0;  // waves of admitted tiles not yet retired
  Arena arena;
  Arena staging;  // pinned host pool
  Clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  // host-memory requests whose results wait for the copy out of pinned
  // staging into the caller's arrays; one thread at a time drains the queue
  // with the lock released (the caller's pages may fault on first touch)
  std::vector<Request*> copyq;
  bool copy_busy = false;
  std::thread thread;
  bool stop = false;
  bool device_error = false;

  uint64_t next_id = 1;
  uint64_t use_clock = 0;
  std::deque<Request*> pending;
  std::vector<Request*> live;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> all;
  std::vector<std::unique_ptr<Resident>> residents;
  // the keyed residents by model key: a lookup per admitted request must not
  // scan every resident model (thousands stay resident in a serving process)
  std::unordered_multimap<uint64_t, Resident*> by_key;
  std::deque<Batch> inflight;
  std::deque<TimedPair> reduce_timing;

  char* staging_block = nullptr;  // the pinned allocation behind `staging`
  char* jobtab_block = nullptr;   // the pinned allocation behind jobtab_host
  // per outstanding batch (slot = batch number % max_inflight): the table of
  // finished requests' records and their summaries, on the device (in the
  // arena) and pinned
  FinEntry* fintab_host = nullptr;
  FinEntry* fintab_dev = nullptr;
  PointSummary* sum_host = nullptr;
  PointSummary* sum_dev = nullptr;
  char* fin_block = nullptr;  // the pinned allocation behind fintab_host, sum_host
  uint64_t batch_seq = 0;
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
  // a queued copy fails with the rest; one that a thread is running (state
  // kCopy, no longer queued) completes, as its results are whole
  for (Request* r : c->copyq) r->state = RState::kPending;
  c->copyq.clear();
  for (auto& kv : c->all) {
    Request* r = kv.second.get();
    if (r->state != RState::kDone && r->state != RState::kFailed && r->state != RState::kCopy) {
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

void release_buf(lti_ctx* c, HostBuf& hb) {
  if (hb.pinned && hb.base) c->staging.release(hb.base, hb.bytes);
  hb.base = nullptr;
  hb.pinned = false;
  hb.fallback.clear();
  hb.fallback.shrink_to_fit();
}

void release_stage(lti_ctx* c, HostStage& hs) {
  release_buf(c, hs.in);
  release_buf(c, hs.out);
}

// Take `bytes` of host memory: pinned when the pool has room; pageable only
// when `may_page` (otherwise nullptr: wait for the pool).
bool take_buf(lti_ctx* c, HostBuf& hb, size_t bytes, bool may_page) {
  hb.bytes = bytes;
  hb.base = static_cast<char*>(c->staging.alloc(bytes));
  hb.pinned = hb.base != nullptr;
  if (hb.pinned) return true;
  if (!may_page) return false;
  try {
    hb.fallback.resize(bytes);
  } catch (...) {
    return false;
  }
  hb.base = hb.fallback.data();
  return true;
}

// Device bytes of a request (besides a shared resident model); the block holds
// [A..D | omega | G | info] (host-memory requests), its own point records
// (device requests without info_out), the refinement queue, then the
// reduction scratch.
struct Need {
  size_t omega = 0, G = 0, info = 0, dG = 0, queue = 0, inputs = 0, work = 0, model = 0;
  size_t block() const { return omega + G + info + dG + queue + inputs + work; }
};

// n, sm, sp: the solved system's sizes.
Need request_need(const lti_request& q, bool needs_model, int sm, int sp) {
  const int n = q.nx, m = q.nu, p = q.ny;
  Need nd;
  if (q.mem == LTI_MEM_HOST) {
    nd.omega = align_up(sizeof(double) * omega_doubles(q));
    nd.G = align_up(sizeof(double) * 2 * (size_t)q.n_omega * p * m);
  }
  if (q.mem == LTI_MEM_HOST || !q.info_out) nd.info = align_up(sizeof(lti_point_info) * q.n_omega);
  if (q.mem == LTI_MEM_HOST && q.dG_out) nd.dG = nd.G;
  // one queue entry per (point, column group) at most; sm groups at most
  nd.queue = align_up(8 + 8 * (size_t)q.n_omega * sm);
  if (needs_model) {
    if (q.mem == LTI_MEM_HOST)  // same per-matrix alignment as the host staging
      nd.inputs = align_up(sizeof(double) * n * n) + align_up(sizeof(double) * n * m) +
                  align_up(sizeof(double) * p * n) + align_up(sizeof(double) * p * m) +
                  (q.E ? align_up(sizeof(double) * n * n) : 0);
    nd.work = q.E ? align_up(reduce_ht_work_bytes(n, sm, sp)) : reduce_work_bytes(n, sm, sp);
    nd.model = align_up(reduced_bytes(n, sm, sp, q.E != nullptr));
  }
  return nd;
}

Resident* find_resident(lti_ctx* c, const Request& r) {
  if (r.req.model_key == 0) return nullptr;
  const auto range = c->by_key.equal_range(r.req.model_key);
  for (auto it = range.first; it != range.second; ++it) {
    Resident* res = it->second;
    if (res->n == r.req.nx && res->m == r.req.nu && res->p == r.req.ny && res->hash == r.hash &&
        res->trans == r.trans && res->desc == (r.req.E ? 1 : 0))
      return res;
  }
  return nullptr;
}

void add_resident(lti_ctx* c, std::unique_ptr<Resident> up) {
  Resident* res = up.get();
  res->slot = c->residents.size();
  c->residents.push_back(std::move(up));
  if (res->key != 0) c->by_key.emplace(res->key, res);
}

// Frees the model's memory and its record (res is invalid afterwards).
void drop_resident(lti_ctx* c, Resident* res) {
  pass_release(c, res->ready);
  c->arena.release(res->block, res->bytes);
  if (res->key != 0) {
    const auto range = c->by_key.equal_range(res->key);
    for (auto it = range.first; it != range.second; ++it) {
      if (it->second == res) {
        c->by_key.erase(it);
        break;
      }
    }
  }
  // swap with the last record and drop it
  const size_t s = res->slot;
  if (s + 1 != c->residents.size()) {
    c->residents[s] = std::move(c->residents.back());
    c->residents[s]->slot = s;
  }
  c->residents.pop_back();
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
    if (r->state == RState::kDone || r->state == RState::kCopy) pass_release(c, res->ready);
    res->refs--;
    r->model = nullptr;
    if (res->key == 0 && res->refs == 0) drop_resident(c, res);
  }
}

// Work collected by one admission pass.
struct PassWork {
  std::vector<ReduceJob> jobs[kNumReduceClasses];
  std::vector<std::pair<uint32_t*, uint32_t>> zero;  // device ranges to clear (words)
  bool copies = false;  // uploads were issued on the admission stream
  size_t total() const {
    size_t t = 0;
    for (const auto& v : jobs) t += v.size();
    return t;
  }
};

bool admit_one(lti_ctx* c, Request* r, PassWork& pw) {
  const lti_request& q = r->req;
  const int n = q.nx, sm = r->sm, sp = r->sp;
  Resident* res = find_resident(c, *r);
  const bool needs_model = (res == nullptr);
  if (needs_model && (int)pw.total() >= kMaxJobs) return false;
  const Need nd = request_need(q, needs_model, sm, sp);
  // pinned host memory for the results (pageable only for results larger
  // than the whole pool), then device memory; a request that does not fit
  // waits
  // (device-memory requests need none: their records stay on the device and
  // the finishing batch summarises them)
  HostStage& hs = r->hs;
  const bool host = q.mem == LTI_MEM_HOST;
  const size_t ibytes = host ? sizeof(lti_point_info) * q.n_omega : 0;
  const size_t gbytes = host ? sizeof(double) * 2 * (size_t)q.n_omega * q.ny * q.nu : 0;
  hs.offG = 0;
  hs.offInfo = align_up(gbytes);
  hs.offDG = hs.offInfo + align_up(ibytes);
  hs.outBytes = !host ? 0 : q.dG_out ? hs.offDG + gbytes : hs.offInfo + ibytes;
  if (hs.outBytes && !take_buf(c, hs.out, hs.outBytes, align_up(hs.outBytes) > c->staging.size())) return false;
  void* mblock = nullptr;
  if (needs_model) {
    mblock = alloc_evicting(c, nd.model);
    if (!mblock) {
      release_buf(c, hs.out);
      return false;
    }
  }
  void* block = alloc_evicting(c, nd.block());
  if (!block) {
    if (mblock) c->arena.release(mblock, nd.model);
    release_buf(c, hs.out);
    return false;
  }
  if (needs_model) {
    auto up = std::make_unique<Resident>();
    res = up.get();
    res->key = q.model_key;
    res->hash = r->hash;
    res->n = n;
    res->m = q.nu;
    res->p = q.ny;
    res->trans = r->trans;
    res->desc = q.E ? 1 : 0;
    res->block = mblock;
    res->bytes = nd.model;
    reduced_layout(mblock, n, sm, sp, r->trans, &res->rm, q.E != nullptr);
    add_resident(c, std::move(up));
    c->stats.reductions++;
  } else {
    c->stats.reduction_cache_hits++;
  }
  res->refs++;
  res->last_use = ++c->use_clock;
  r->model = res;
  r->reused = !needs_model;
  // what the request's sweeps have to wait for: its own pass (uploads, the
  // cleared queue) and the pass that reduces its model
  if (needs_model) res->ready = pass_ref(c->pass);
  r->ready = pass_ref(c->pass);
  if (!needs_model) r->model_ready = pass_ref(res->ready);
  r->block = block;
  r->block_bytes = nd.block();

  char* b = static_cast<char*>(block);
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
    job.E = q.E;
  }
  if (host) {
    // A..D (when this request reduces its model) and omega sit back to back
    // in staging; the block mirrors that layout, so one H2D copy moves them
    const size_t src0 = needs_model ? hs.offA : hs.offW;
    const size_t bytes = hs.offW - src0 + sizeof(double) * omega_doubles(q);
    e = hipMemcpyAsync(b, hs.in.base + src0, bytes, hipMemcpyHostToDevice, c->rstream);
    pw.copies = true;
    if (needs_model) {
      job.A = reinterpret_cast<const double*>(b);
      job.B = reinterpret_cast<const double*>(b + (hs.offB - hs.offA));
      job.C = reinterpret_cast<const double*>(b + (hs.offC - hs.offA));
      job.D = reinterpret_cast<const double*>(b + (hs.offD - hs.offA));
      if (q.E) job.E = reinterpret_cast<const double*>(b + (hs.offE - hs.offA));
    }
    b += nd.inputs;
    d_omega = reinterpret_cast<const double*>(b);
    b += nd.omega;
    r->dOffG = (size_t)(b - static_cast<char*>(block));
    d_G = reinterpret_cast<double*>(b);
    b += nd.G;
  }
  if (nd.info) {
    d_info = reinterpret_cast<lti_point_info*>(b);
    b += nd.info;
  }
  double* d_dG = q.dG_out;
  if (nd.dG) {  // host requests: right after the records, as in staging
    d_dG = reinterpret_cast<double*>(b);
    b += nd.dG;
  }
  r->dinfo = d_info;
  uint32_t* fbq = reinterpret_cast<uint32_t*>(b);
  b += nd.queue;
  pw.zero.emplace_back(fbq, 1u);
  if (needs_model) {
    job.out = res->rm;
    job.work = nd.work ? reinterpret_cast<double*>(b) : nullptr;
    b += nd.work;
    pw.jobs[q.E ? kReduceHT : reduce_class(n, sm, sp)].push_back(job);
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
  desc.dG = d_dG;
  desc.T = res->rm.T;
  desc.info = d_info;
  desc.fbq = fbq;
  desc.n = n;
  desc.m = sm;
  desc.p = sp;
  desc.precision = q.precision;
  desc.rtol = q.rtol;
  desc.flags = (r->trans ? kFlagTrans : 0u) | ((c->flags & LTI_CFG_FORCE_DD) ? kFlagForceDD : 0u) |
               (q.E ? kFlagDescriptor : 0u) | ((uint32_t)q.points << 8);
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return true;
  }
  r->K = q.n_omega;
  TileKnobs kn;
  kn.tile_points = c->tile_points;
  kn.rhs_split = c->rhs_split;
  kn.use_sweep16 = c->use_sweep16;
  kn.use_sweep32 = c->use_sweep32;
  kn.sweep32_max_cols = c->sweep32_max_cols;
  kn.descriptor = q.E != nullptr;
  const TilePlan tp = plan_tiles(q.precision, n, sm, sp, r->K, std::max<int64_t>(0, c->target_tiles16 - c->outstanding_waves),
                                 std::max<int64_t>(0, c->target_tiles - c->outstanding_waves), kn);
  r->F = tp.F;
  r->S = tp.S;
  r->mc = tp.mc;
  r->kclass = tp.kclass;
  // several column groups per point: their records are merged (cleared first)
  if (r->S > 1) {
    desc.flags |= kFlagMergeInfo;
    pw.zero.emplace_back(reinterpret_cast<uint32_t*>(d_info), (uint32_t)(2 * r->K));
  }
  r->stage = tp.stage;
  r->ntiles = tp.ntiles;
  r->waves_per_tile = tp.waves_per_tile;
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
  PassWork pw;
  // with no sweeps outstanding the pass goes on the sweep stream, which
  // orders the two without a cross-stream wait
  c->rstream = c->inflight.empty() ? c->stream : c->rstreams[rs];
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
    if (!admit_one(c, r, pw)) break;
    c->pending.pop_front();
    if (r->state == RState::kLive) c->live.push_back(r);
  }
  if (c->device_error || (pw.total() == 0 && !pw.copies && pw.zero.empty())) return;
  c->next_rstream = (rs + 1) % c->n_rstreams;
  hipError_t e = hipSuccess;
  // the cleared queues and records (before any kernel of these requests)
  ZeroLaunch Z;
  for (size_t i0 = 0; i0 < pw.zero.size() && e == hipSuccess; i0 += kMaxZero) {
    Z.n = (int)std::min<size_t>(kMaxZero, pw.zero.size() - i0);
    for (int i = 0; i < Z.n; ++i) {
      Z.e[i].p = pw.zero[i0 + i].first;
      Z.e[i].words = pw.zero[i0 + i].second;
    }
    e = launch_zero(Z, c->rstream);
  }
  const bool timed = (c->flags & LTI_CFG_KERNEL_TIMING) != 0 && pw.total() > 0;
  TimedPair tp{nullptr, nullptr};
  if (timed && e == hipSuccess) {
    tp.a = get_event(c, true);
    tp.b = get_event(c, true);
    e = hipEventRecord(tp.a, c->rstream);
  }
  // the pass's jobs go to the device as one table (this admission stream's:
  // its previous pass has completed), one launch per kernel class
  if (pw.total() > 0 && e == hipSuccess) {
    ReduceJob* th = c->jobtab_host[rs];
    ReduceJob* td = c->jobtab_dev[rs];
    size_t o = 0;
    size_t first[kNumReduceClasses];
    for (int rc = 0; rc < kNumReduceClasses; ++rc) {
      first[rc] = o;
      std::copy(pw.jobs[rc].begin(), pw.jobs[rc].end(), th + o);
      o += pw.jobs[rc].size();
    }
    e = hipMemcpyAsync(td, th, o * sizeof(ReduceJob), hipMemcpyHostToDevice, c->rstream);
    for (int rc = 0; rc < kNumReduceClasses && e == hipSuccess; ++rc) {
      if (pw.jobs[rc].empty()) continue;
      ReduceLaunch L{td + first[rc], th + first[rc], (int)pw.jobs[rc].size()};
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

// Copy a finished host-memory request's results to its pinned staging: G
// and its records (and dG) in one copy, back to back in the block and in
// staging (same offsets).  Device-memory requests copy nothing.
hipError_t copy_results(lti_ctx* c, Request* r, hipStream_t s) {
  (void)c;
  if (r->req.mem != LTI_MEM_HOST) return hipSuccess;
  HostStage& hs = r->hs;
  const char* src = static_cast<const char*>(r->block) + r->dOffG;
  return hipMemcpyAsync(hs.out.base + hs.offG, src, hs.outBytes, hipMemcpyDeviceToHost, s);
}

// Gather up to batch_tiles tiles from the live requests (oldest first) into
// one batch: one launch per kernel class and kMaxSegs requests, each request
// a contiguous range of its tiles.  Requests whose last tiles are in the
// batch are finished in it: refinement of their queued points, result copy.
void launch(lti_ctx* c) {
  if (c->live.empty() || (int)c->inflight.size() >= c->max_inflight) return;
  constexpr int kAllClasses = kAllSweepClasses;
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
  std::vector<Request*> fin;  // requests whose last tiles are in this batch
  for (Request* r : c->live) {
    if (total >= c->batch_tiles || (int)fin.size() >= kMaxFin) break;
    if (r->state != RState::kLive || r->next_tile >= r->ntiles) continue;
    if (!eligible(r)) continue;
    const int64_t take = std::min<int64_t>(r->ntiles - r->next_tile, c->batch_tiles - total);
    per[r->kclass].push_back(Piece{r, r->next_tile, take});
    lds[r->kclass] = std::max(lds[r->kclass], r->stage);
    r->next_tile += take;
    total += take;
    b.credit.emplace_back(r, take);
    if (r->next_tile == r->ntiles) fin.push_back(r);
    if (r->res.t_first_launch_us == 0.0) r->res.t_first_launch_us = c->now_us();
  }
  if (total == 0) return;
  hipError_t e = hipSuccess;
  const bool timed = (c->flags & LTI_CFG_KERNEL_TIMING) != 0;
  // the batch's launches: per kernel class, kMaxSegs requests each, with an
  // estimate of their work (tiles x n^2 x (columns + 2)) for balancing
  struct Job {
    int k;
    size_t lds;
    SweepLaunch L;
    double work;
  };
  std::vector<Job> jobs;
  for (int k = 0; k < kAllClasses; ++k) {
    const std::vector<Piece>& v = per[k];
    for (size_t i0 = 0; i0 < v.size(); i0 += kMaxSegs) {
      Job jb;
      jb.k = k;
      jb.lds = c->stage_lds ? lds[k] : 0;
      jb.work = 0.0;
      SweepLaunch& L = jb.L;
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
        const double n = pc.r->req.nx;
        jb.work += (double)pc.count * pc.r->F * n * n * (pc.r->mc + 2.0);
      }
      L.ntiles = (int)t;
      jobs.push_back(jb);
    }
  }
  // largest first, each to the least loaded sweep stream.  The streams are
  // not joined between batches: a stream whose share of this batch is done
  // goes on with the next batch's launches while the others finish.
  std::sort(jobs.begin(), jobs.end(), [](const Job& x, const Job& y) { return x.work > y.work; });
  const int ns = jobs.size() > 1 ? c->n_sweep_streams : 1;
  hipStream_t streams[kMaxSweepStreams] = {c->stream, c->aux[0], c->aux[1]};
  double load[kMaxSweepStreams] = {0.0, 0.0, 0.0};
  std::vector<int> on(jobs.size());
  bool used[kMaxSweepStreams] = {false, false, false};
  for (size_t q = 0; q < jobs.size(); ++q) {
    int si = 0;
    for (int i = 1; i < ns; ++i)
      if (load[i] < load[si]) si = i;
    load[si] += jobs[q].work;
    on[q] = si;
    used[si] = true;
  }
  // each stream used first waits for the uploads and reductions the batch's
  // requests depend on (passes on that stream itself are ordered by it)
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    if (!used[i]) continue;
    std::vector<const PassEvent*> waited;
    for (auto& cr : b.credit)
      for (const PassEvent* pe : {cr.first->ready, cr.first->model_ready})
        if (pe && pe->stream != streams[i] && !pass_done(pe) &&
            std::find(waited.begin(), waited.end(), pe) == waited.end()) {
          waited.push_back(pe);
          if (e == hipSuccess) e = hipStreamWaitEvent(streams[i], pe->ev, 0);
        }
    if (timed && e == hipSuccess) {
      hipEvent_t ev = get_event(c, true);
      e = ev ? hipEventRecord(ev, streams[i]) : hipErrorOutOfMemory;
      if (ev) b.tstart.push_back(ev);
    }
  }
  for (size_t q = 0; q < jobs.size() && e == hipSuccess; ++q) {
    e = launch_any_sweep(jobs[q].k, jobs[q].L, jobs[q].lds, streams[on[q]]);
    c->stats.sweep_launches++;
  }
  // The finishing stream waits for the batch's sweeps on every stream used.
  // A batch on one sweep stream while every earlier batch has retired
  // finishes on that stream itself: nothing else can be outstanding, and a
  // short request then makes no cross-stream hop.
  const int64_t seq = (int64_t)c->batch_seq;
  int n_used = 0, only = 0;
  for (int i = 0; i < ns; ++i)
    if (used[i]) {
      ++n_used;
      only = i;
    }
  bool inline_finish = n_used == 1;
  for (int i = 0; i <= kMaxSweepStreams && inline_finish; ++i)
    if (i != only && c->last_use[i] >= c->batches_retired) inline_finish = false;
  hipStream_t fs = inline_finish ? streams[only] : c->fstream;
  for (int i = 0; i < ns; ++i)
    if (used[i]) c->last_use[i] = seq;
  if (!inline_finish) c->last_use[kMaxSweepStreams] = seq;
  b.joins_timed = timed;
  for (int i = 0; i < ns && e == hipSuccess; ++i) {
    if (!used[i] || (inline_finish && !timed)) continue;
    hipEvent_t join = get_event(c, timed);
    if (!join) {
      e = hipErrorOutOfMemory;
      break;
    }
    b.joins.push_back(join);
    e = hipEventRecord(join, streams[i]);
    if (e == hipSuccess && !inline_finish) e = hipStreamWaitEvent(fs, join, 0);
  }
  auto time_mark = [&](int fam) {
    if (!timed || e != hipSuccess) return;
    hipEvent_t ev = get_event(c, true);
    if (!ev) {
      e = hipErrorOutOfMemory;
      return;
    }
    e = hipEventRecord(ev, fs);
    b.tev.push_back(ev);
    if (fam >= 0) b.tfam.push_back(fam);
  };
  // finish the requests whose last tiles are in the batch: the extended
  // refinement of their queued points (the grid is sized by their points; a
  // workgroup that finds the queues empty exits at once), then the results
  // to host memory.  Their earlier tiles, in earlier batches, are done: the
  // finishing stream runs the batches' finishing work in order.
  if (!fin.empty() && e == hipSuccess) {
    time_mark(-1);
    DDLaunch D;
    for (size_t i0 = 0; i0 < fin.size() && e == hipSuccess; i0 += kMaxDDSegs) {
      D.nseg = (int)std::min<size_t>(kMaxDDSegs, fin.size() - i0);
      int64_t pts = 0;
      for (int i = 0; i < D.nseg; ++i) {
        Request* r = fin[i0 + i];
        D.seg[i].rd = r->desc;
        D.seg[i].rm = r->model->rm;
        D.seg[i].K = (uint64_t)r->K;
        pts += r->K * r->S;
      }
      // at most one workgroup per CU: the kernel's registers allow one
      // resident workgroup per CU, so a larger grid adds only dispatches
      // (every launch pays them, and most find their queues empty)
      const int grid = (int)std::max<int64_t>(16, std::min<int64_t>(c->n_cus, pts / 32));
      e = launch_refine_dd(D, grid, fs);
    }
    time_mark(LTI_KF_REFINE_DD);
    // the summaries of their point records: one table up, one kernel, one
    // copy down (this batch's slot; the batch that used it last has retired)
    const size_t slot = (size_t)(c->batch_seq % (uint64_t)c->max_inflight) * kMaxFin;
    FinEntry* th = c->fintab_host + slot;
    for (size_t i = 0; i < fin.size(); ++i) {
      th[i].info = fin[i]->dinfo;
      th[i].K = (uint64_t)fin[i]->K;
      fin[i]->sum = c->sum_host + slot + i;
    }
    const int nf = (int)fin.size();
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->fintab_dev + slot, th, sizeof(FinEntry) * nf, hipMemcpyHostToDevice, fs);
    if (e == hipSuccess) e = launch_summarize(c->fintab_dev + slot, c->sum_dev + slot, nf, fs);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->sum_host + slot, c->sum_dev + slot, sizeof(PointSummary) * nf, hipMemcpyDeviceToHost,
                         fs);
    for (size_t i = 0; i < fin.size() && e == hipSuccess; ++i) e = copy_results(c, fin[i], fs);
  }
  c->batch_seq++;
  b.done = get_event(c, false);
  if (e == hipSuccess) e = b.done ? hipEventRecord(b.done, fs) : hipErrorOutOfMemory;
  c->stats.tiles_launched += total;
  if (e != hipSuccess) {
    fail_all(c, LTI_EDEVICE);
    return;
  }
  c->inflight.push_back(std::move(b));
}

// Results are in pinned staging (the batch that finished the request copied
// them there): hand them to the caller and count the point records.
// The copy of a host-memory request's results from pinned staging into the
// caller's arrays (no context state: runs with the lock released).
void copy_to_caller(const Request* r) {
  const lti_request& q = r->req;
  const HostStage& hs = r->hs;
  std::memcpy(q.G_out, hs.out.base + hs.offG, sizeof(double) * 2 * (size_t)q.n_omega * q.ny * q.nu);
  if (q.info_out) std::memcpy(q.info_out, hs.out.base + hs.offInfo, sizeof(lti_point_info) * q.n_omega);
  if (q.dG_out) std::memcpy(q.dG_out, hs.out.base + hs.offDG, sizeof(double) * 2 * (size_t)q.n_omega * q.ny * q.nu);
}

// Last step of a completed request (lock held): its staging goes back to the
// pool and poll() sees it done.
void finish_request(lti_ctx* c, Request* r) {
  release_stage(c, r->hs);
  if (r->state == RState::kFailed) return;  // failed meanwhile (fail_all)
  r->res.t_done_us = c->now_us();
  r->state = RState::kDone;
  c->stats.requests_done++;
  c->stats.points_done += r->req.n_omega;
}

// Copies of the queued requests, with the lock released while they run;
// callers hold `lk`, which is held again on return.  A thread that finds
// another one draining returns at once (that one takes the new entries too).
void drain_copies(lti_ctx* c, std::unique_lock<std::mutex>& lk) {
  if (c->copy_busy || c->copyq.empty()) return;
  c->copy_busy = true;
  while (!c->copyq.empty()) {
    std::vector<Request*> work;
    work.swap(c->copyq);
    lk.unlock();
    for (const Request* r : work) copy_to_caller(r);
    lk.lock();
    for (Request* r : work) finish_request(c, r);
    c->cv_done.notify_all();
  }
  c->copy_busy = false;
}

void complete_request(lti_ctx* c, Request* r) {
  const lti_request& q = r->req;
  r->res.status = LTI_OK;
  r->res.n_points = q.n_omega;
  const PointSummary& ps = *r->sum;
  r->res.n_refined = ps.count[LTI_PATH_REFINED];
  r->res.n_fallback = ps.count[LTI_PATH_FALLBACK];
  r->res.n_singular = ps.count[LTI_PATH_SINGULAR];
  r->res.n_fp64_dd = ps.count[LTI_PATH_FP64_DD];
  r->res.max_est_rel_err = std::max(0.0, (double)ps.max_est);
  if (q.mem == LTI_MEM_HOST) {
    r->state = RState::kCopy;
    c->copyq.push_back(r);
  } else {
    finish_request(c, r);
  }
  release_request_memory(c, r);  // the device side is done either way
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
  while (!c->inflight.empty()) {
    Batch& b = c->inflight.front();
    const hipError_t q = hipEventQuery(b.done);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) {
      fail_all(c, LTI_EDEVICE);
      return true;
    }
    if (!b.tev.empty()) {
      for (size_t i = 0; i + 1 < b.tev.size() && i < b.tfam.size(); ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, b.tev[i], b.tev[i + 1]) != hipSuccess) continue;
        const int f = b.tfam[i];
        c->stats.family_ms[f] += ms;
        c->stats.family_launches[f]++;
      }
      for (hipEvent_t ev : b.tev) put_event(c, ev, true);
      b.tev.clear();
    }
    if (!b.tstart.empty() && b.joins_timed && !b.joins.empty()) {
      // the batch's sweep interval, from its first start to its last join,
      // counted where it goes past the end of the batches retired before
      // (batches overlap on the streams): times relative to tstart[0]
      float lo = 0.f, hi = 0.f, ms = 0.f;
      bool ok = true;
      for (hipEvent_t ev : b.tstart) {
        ok = ok && hipEventElapsedTime(&ms, b.tstart[0], ev) == hipSuccess;
        lo = std::min(lo, ms);
      }
      size_t last = 0;
      for (size_t i = 0; i < b.joins.size(); ++i) {
        ok = ok && hipEventElapsedTime(&ms, b.tstart[0], b.joins[i]) == hipSuccess;
        if (i == 0 || ms > hi) {
          hi = ms;
          last = i;
        }
      }
      float from = lo;
      if (ok && c->union_end && hipEventElapsedTime(&ms, b.tstart[0], c->union_end) == hipSuccess)
        from = std::max(from, ms);
      if (ok) {
        if (hi > from) c->stats.sweep_kernel_ms += hi - from;
        c->stats.timed_sweep_launches++;
        if (!c->union_end || hi > from) {
          // the batch's last join becomes the new end of the union
          if (c->union_end) put_event(c, c->union_end, true);
          c->union_end = b.joins[last];
          b.joins[last] = nullptr;
        }
      }
      for (hipEvent_t ev : b.tstart) put_event(c, ev, true);
      b.tstart.clear();
    }
    for (auto& cr : b.credit) {
      Request* r = cr.first;
      r->tiles_done += cr.second;
      c->outstanding_waves -= cr.second * r->waves_per_tile;
      if (r->tiles_done == r->ntiles && r->state == RState::kLive) complete_request(c, r);
    }
    put_event(c, b.done, false);
    for (hipEvent_t ev : b.joins)
      if (ev) put_event(c, ev, b.joins_timed);
    c->inflight.pop_front();
    c->batches_retired++;
    progressed = true;
  }
  // completed requests leave the live list here, those with a copy still to
  // run included (the copy queue holds them; poll() may free a request as
  // soon as it is done, so nothing else may keep a pointer to it)
  for (auto it = c->live.begin(); it != c->live.end();) {
    Request* r = *it;
    if (r->state == RState::kDone || r->state == RState::kFailed || r->state == RState::kCopy) {
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
  for (int i = 0; i + 1 < kMaxSweepStreams; ++i) {
    if (c->aux[i]) (void)hipStreamDestroy(c->aux[i]);
    c->aux[i] = nullptr;
  }
  if (c->fstream) (void)hipStreamDestroy(c->fstream);
  c->fstream = nullptr;
}

bool busy(const lti_ctx* c) {
  return !c->inflight.empty() || !c->live.empty() || !c->reduce_timing.empty() || !c->pending.empty() ||
         !c->copyq.empty();
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
    const bool progressed = pump(c);
    drain_copies(c, lk);
    if (progressed) {
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
  if (q->points != LTI_POINTS_JW && q->points != LTI_POINTS_S && q->points != LTI_POINTS_Z) return LTI_EINVAL;
  if (q->n_omega > (int64_t)UINT32_MAX) return LTI_EINVAL;
  if (std::isnan(q->rtol) || q->rtol >= 1.0) return LTI_EINVAL;
  if (q->nx > kMaxNWG || q->nu > kMaxRhs || q->ny > kMaxRhs) return LTI_EUNSUPPORTED;
  // descriptor systems: float64 one-frequency kernels (n <= kMaxN), no
  // derivative
  if (q->E && (q->nx > kMaxN || q->dG_out)) return LTI_EUNSUPPORTED;
  // tile indices (at most n_omega x nu per request) are 32-bit
  if (q->n_omega * q->nu > (int64_t)UINT32_MAX) return LTI_EUNSUPPORTED;
  return LTI_OK;
}

// Stage a host-memory request's inputs in `hs.in` (pinned when the pool has
// room, else pageable: the H2D copy is then a synchronous one).
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
  hs.offE = take(q.E ? sizeof(double) * n * n : 0);
  hs.offW = take(sizeof(double) * omega_doubles(q));
  bool ok;
  {
    std::lock_guard<std::mutex> lk(c->mu);
    ok = take_buf(c, hs.in, off, true);
  }
  if (!ok) return LTI_ENOMEM;
  char* base = hs.in.base;
  // A..D must be contiguous in this order (one H2D copy)
  std::memcpy(base + hs.offA, q.A, sizeof(double) * n * n);
  std::memcpy(base + hs.offB, q.B, sizeof(double) * n * m);
  std::memcpy(base + hs.offC, q.C, sizeof(double) * p * n);
  if (q.D)
    std::memcpy(base + hs.offD, q.D, sizeof(double) * p * m);
  else
    std::memset(base + hs.offD, 0, sizeof(double) * p * m);
  if (q.E) std::memcpy(base + hs.offE, q.E, sizeof(double) * n * n);
  std::memcpy(base + hs.offW, q.omega, sizeof(double) * omega_doubles(q));
  // the model's identity: its dimensions and the bytes of A, B, C, D (not
  // the alignment gaps between them in staging, which hold whatever the
  // pool held before); only keyed requests are ever matched
  r->hash = 0;
  if (q.model_key == 0) return LTI_OK;
  uint64_t h = 1469598103934665603ull;
  const int dims[3] = {n, m, p};
  h = fnv1a(dims, sizeof(dims), h);
  h = fnv1a(base + hs.offA, sizeof(double) * n * n, h);
  h = fnv1a(base + hs.offB, sizeof(double) * n * m, h);
  h = fnv1a(base + hs.offC, sizeof(double) * p * n, h);
  h = fnv1a(base + hs.offD, sizeof(double) * p * m, h);
  if (q.E) h = fnv1a(base + hs.offE, sizeof(double) * n * n, h);
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
  if (const char* e = std::getenv("LTI_FREQRESP_TILE_POINTS")) c->tile_points = std::max(0, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_TARGET_TILES")) c->target_tiles = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_STAGE_LDS")) c->stage_lds = std::atoi(e) != 0;
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP16")) c->use_sweep16 = std::atoi(e) != 0;
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP32")) c->use_sweep32 = std::atoi(e) != 0;
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP32_COLS"))
    c->sweep32_max_cols = std::max(1, std::min(kMaxRhs, std::atoi(e)));
  if (const char* e = std::getenv("LTI_FREQRESP_TARGET_TILES16")) c->target_tiles16 = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_MAX_INFLIGHT"))
    c->max_inflight = std::max(1, std::min(64, std::atoi(e)));
  if (const char* e = std::getenv("LTI_FREQRESP_ADMIT_STREAMS"))
    c->n_rstreams = std::max(1, std::min(kAdmitStreams, std::atoi(e)));
  if (const char* e = std::getenv("LTI_FREQRESP_BATCH_TILES")) c->batch_tiles = std::max(1, std::atoi(e));
  if (const char* e = std::getenv("LTI_FREQRESP_SWEEP_STREAMS"))
    c->n_sweep_streams = std::max(1, std::min(kMaxSweepStreams, std::atoi(e)));
  c->t0 = Clock::now();
  if (hipSetDevice(c->device) != hipSuccess) return LTI_EDEVICE;
  // the arena, minus the reduction job tables (one per admission stream) and
  // the finished-request tables and summaries (one slot per outstanding
  // batch)
  const size_t tab_bytes = align_up(sizeof(ReduceJob) * kMaxJobs);
  const size_t fin_slots = (size_t)c->max_inflight * kMaxFin;
  const size_t fintab_bytes = align_up(sizeof(FinEntry) * fin_slots);
  const size_t sum_bytes = align_up(sizeof(PointSummary) * fin_slots);
  const size_t reserved = kAdmitStreams * tab_bytes + fintab_bytes + sum_bytes;
  if (cfg->arena_bytes < reserved + (size_t(1) << 20)) return LTI_EINVAL;
  char* abase = static_cast<char*>(cfg->arena);
  for (int i = 0; i < kAdmitStreams; ++i) c->jobtab_dev[i] = reinterpret_cast<ReduceJob*>(abase + i * tab_bytes);
  c->fintab_dev = reinterpret_cast<FinEntry*>(abase + kAdmitStreams * tab_bytes);
  c->sum_dev = reinterpret_cast<PointSummary*>(abase + kAdmitStreams * tab_bytes + fintab_bytes);
  c->arena.init(abase + reserved, cfg->arena_bytes - reserved);
  const size_t staging = cfg->host_staging_bytes ? cfg->host_staging_bytes : kDefaultStaging;
  void* hp = nullptr;
  if (hipHostMalloc(&hp, staging, hipHostMallocDefault) != hipSuccess) return LTI_EDEVICE;
  c->staging_block = static_cast<char*>(hp);
  c->staging.init(c->staging_block, staging);
  void* jp = nullptr;
  if (hipHostMalloc(&jp, kAdmitStreams * tab_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipHostFree(hp);
    return LTI_EDEVICE;
  }
  c->jobtab_block = static_cast<char*>(jp);
  for (int i = 0; i < kAdmitStreams; ++i)
    c->jobtab_host[i] = reinterpret_cast<ReduceJob*>(c->jobtab_block + i * tab_bytes);
  void* fp = nullptr;
  if (hipHostMalloc(&fp, fintab_bytes + sum_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipHostFree(hp);
    (void)hipHostFree(jp);
    return LTI_EDEVICE;
  }
  c->fin_block = static_cast<char*>(fp);
  c->fintab_host = reinterpret_cast<FinEntry*>(c->fin_block);
  c->sum_host = reinterpret_cast<PointSummary*>(c->fin_block + fintab_bytes);
  auto free_host = [&] {
    (void)hipHostFree(hp);
    (void)hipHostFree(jp);
    (void)hipHostFree(fp);
  };
  // tuning knob (not part of the ABI): keep the sweeps off the first N CUs,
  // so that reductions always find room beside them
  int reserved_cus = kReservedCUs;
  if (const char* e = std::getenv("LTI_FREQRESP_RESERVED_CUS")) reserved_cus = std::max(0, std::atoi(e));
  // a sweep stream: on every CU but the first reserved_cus, when reserving
  std::vector<uint32_t> sweep_mask;
  {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess && ncu > 0)
      c->n_cus = ncu;
    if (reserved_cus > 0 &&
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, c->device) == hipSuccess &&
        reserved_cus < ncu) {
      sweep_mask.assign((ncu + 31) / 32, 0u);
      for (int cu = reserved_cus; cu < ncu; ++cu) sweep_mask[cu / 32] |= 1u << (cu % 32);
    }
  }
  auto make_sweep_stream = [&](hipStream_t* st) {
    if (!sweep_mask.empty()) return hipExtStreamCreateWithCUMask(st, (uint32_t)sweep_mask.size(), sweep_mask.data());
    return hipStreamCreateWithFlags(st, hipStreamNonBlocking);
  };
  if (cfg->stream) {
    c->stream = static_cast<hipStream_t>(cfg->stream);
  } else {
    const hipError_t e = make_sweep_stream(&c->stream);
    if (e != hipSuccess) {
      free_host();
      return LTI_EDEVICE;
    }
    c->own_stream = true;
  }
  bool ok = true;
  for (int i = 0; i < c->n_rstreams && ok; ++i)
    ok = hipStreamCreateWithFlags(&c->rstreams[i], hipStreamNonBlocking) == hipSuccess;
  for (int i = 0; i + 1 < c->n_sweep_streams && ok; ++i) ok = make_sweep_stream(&c->aux[i]) == hipSuccess;
  if (ok) ok = hipStreamCreateWithFlags(&c->fstream, hipStreamNonBlocking) == hipSuccess;
  if (!ok) {
    destroy_admit_streams(c.get());
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    free_host();
    return LTI_EDEVICE;
  }
  try {
    c->thread = std::thread(scheduler, c.get());
  } catch (...) {
    free_host();
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
        (q->D && !all_finite(q->D, (size_t)p * m)) || (q->E && !all_finite(q->E, (size_t)n * n)) ||
        !all_finite(q->omega, omega_doubles(*q)))
      return LTI_EINVAL;
  }
  std::unique_ptr<Request> r(new (std::nothrow) Request());
  if (!r) return LTI_ENOMEM;
  r->req = *q;
  if (q->rtol <= 0.0) r->req.rtol = 1e-10;
  if (q->dG_out || q->E) r->req.precision = LTI_PREC_FP64;  // derivatives, descriptors: float64 path
  // fewer outputs than inputs: solve the transposed system, whose
  // right-hand sides are the min(nu, ny) outputs
  r->trans = (p < m && !(c->flags & LTI_CFG_NO_TRANSPOSE)) ? 1 : 0;
  r->sm = r->trans ? p : m;
  r->sp = r->trans ? m : p;
  {
    // checked before staging (the pinned pool is not taken for a request
    // that can never run)
    std::lock_guard<std::mutex> lk(c->mu);
    if (c->device_error) return LTI_EDEVICE;
    const Need nd = request_need(r->req, true, r->sm, r->sp);
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
        drain_copies(c, lk);
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
  for (hipStream_t as : c->aux)
    if (as) (void)hipStreamSynchronize(as);
  (void)hipStreamSynchronize(c->stream);
  if (c->fstream) (void)hipStreamSynchronize(c->fstream);
  for (auto& b : c->inflight) {
    put_event(c, b.done, false);
    for (hipEvent_t ev : b.tev) put_event(c, ev, true);
    for (hipEvent_t ev : b.tstart) put_event(c, ev, true);
    for (hipEvent_t ev : b.joins)
      if (ev) put_event(c, ev, b.joins_timed);
  }
  if (c->union_end) put_event(c, c->union_end, true);
  for (auto& tp : c->reduce_timing) {
    put_event(c, tp.a, true);
    put_event(c, tp.b, true);
  }
  for (PassEvent*& lp : c->last_pass) lp = nullptr;
  for (PassEvent* pe : c->pass_events) {
    put_event(c, pe->ev, false);
    delete pe;
  }
  c->pass_events.clear();
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->timing_pool) (void)hipEventDestroy(e);
  if (c->staging_block) (void)hipHostFree(c->staging_block);
  if (c->jobtab_block) (void)hipHostFree(c->jobtab_block);
  if (c->fin_block) (void)hipHostFree(c->fin_block);
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
    // the most recently used model of this key and these sizes
    const auto range = c->by_key.equal_range(key);
    for (auto it = range.first; it != range.second; ++it) {
      Resident* res = it->second;
      if (res->n == nx && res->m == nu && res->p == ny && (!held || res->last_use > held->last_use)) held = res;
    }
    if (!held) return LTI_ENOENT;
    rm = held->rm;
    held->refs++;
  }
  const int n = nx, sm = rm.m, sp = rm.p;  // the solved system's sizes
  std::vector<double> hp((size_t)hlen(n)), bt((size_t)n * sm), ct((size_t)n * sp);
  hipError_t e = hipSetDevice(c->device);
  for (hipStream_t rs : c->rstreams)
    if (e == hipSuccess && rs) e = hipStreamSynchronize(rs);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess) e = hipMemcpy(hp.data(), rm.H, hp.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(bt.data(), rm.Bt, bt.size() * 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(ct.data(), rm.Ct, ct.size() * 8, hipMemcpyDeviceToHost);
  {
    std::lock_guard<std::mutex> lk(c->mu);
    held->refs--;
  }
  if (e != hipSuccess) return LTI_EDEVICE;
  // Stored: Hs = Qs^T As Qs (packed), Bts = Qs^T Bs (n x sm), Cts = (Cs Qs)^T
  // (n x sp).  Without transposition (As, Bs, Cs) = (A, B, C).  With it,
  // (As, Bs, Cs) = (A^T, C^T, B^T), and the reduction of the model itself is
  // H = Hs^T (lower Hessenberg), Q^T B = (Cs Qs)^T, C Q = (Qs^T Bs)^T.
  auto hs = [&](int i, int j) { return (i <= j + 1) ? hp[hoff(j) + i] : 0.0; };
  if (H) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) H[(size_t)i * n + j] = rm.trans ? hs(j, i) : hs(i, j);
  }
  if (Bt) {
    if (rm.trans)
      std::memcpy(Bt, ct.data(), ct.size() * 8);  // n x sp = n x nu
    else
      std::memcpy(Bt, bt.data(), bt.size() * 8);
  }
  if (Ct) {
    if (rm.trans) {
      for (int a = 0; a < ny; ++a)
        for (int i = 0; i < n; ++i) Ct[(size_t)a * n + i] = bt[(size_t)i * sm + a];
    } else {
      for (int a = 0; a < ny; ++a)
        for (int i = 0; i < n; ++i) Ct[(size_t)a * n + i] = ct[(size_t)i * sp + a];
    }
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
