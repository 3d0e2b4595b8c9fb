// Host-only implementation of the fake HIP runtime (see
// fake_hip/hip/hip_runtime.h) and of the kernel entry points the runtime
// launches, as no-op executors: test infrastructure for running the serving
// runtime's scheduler on the CPU under sanitizers.
//
// Kernel stand-ins: a reduction copies D into the reduced model; a sweep
// writes, for every (point k, column j) of its tiles and every output row a,
//     G(a, j) = D(a, j) + w_k (1 + a + 10 j) + j 0.5 w_k,
// (w_k the first double of point k's omega entry) at the output index of the
// solved system (transposed when the request is), and the point record
// {est = 0, iters = 1 + j0, path = 1}, merged by maximum like the device's;
// the refinement kernel finds every queue empty.  The harness checks that
// every request got exactly its own results.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>

#include "lti_kernels.h"

struct FakeEvent {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0;  // records issued
  uint64_t reached = 0;   // records the stream has reached
};

struct FakeStream {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  bool busy = false;
  bool stop = false;
  std::thread worker;
  FakeStream() {
    worker = std::thread([this] {
      std::unique_lock<std::mutex> lk(mu);
      for (;;) {
        cv.wait(lk, [&] { return stop || !q.empty(); });
        if (q.empty() && stop) return;
        auto op = std::move(q.front());
        q.pop_front();
        busy = true;
        lk.unlock();
        // a little latency, so that the scheduler sees work in flight
        if (std::rand() % 4 == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        op();
        lk.lock();
        busy = false;
        cv.notify_all();
      }
    });
  }
  void push(std::function<void()> f) {
    std::lock_guard<std::mutex> lk(mu);
    q.push_back(std::move(f));
    cv.notify_all();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    cv.wait(lk, [&] { return q.empty() && !busy; });
  }
  ~FakeStream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      stop = true;
      cv.notify_all();
    }
    worker.join();
  }
};

hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  *v = 256;
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = new FakeStream();
  return hipSuccess;
}
hipError_t hipExtStreamCreateWithCUMask(hipStream_t* s, uint32_t, const uint32_t*) {
  return hipStreamCreateWithFlags(s, 0);
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete s;
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
  s->sync();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = new FakeEvent();
  return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = ++e->recorded;
  }
  s->push([e, gen] {
    std::lock_guard<std::mutex> lk(e->mu);
    if (e->reached < gen) e->reached = gen;
    e->cv.notify_all();
  });
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(e->mu);
  return e->reached >= e->recorded ? hipSuccess : hipErrorNotReady;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.01f;
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = e->recorded;
  }
  s->push([e, gen] {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&] { return e->reached >= gen; });
  });
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
  s->push([=] { std::memcpy(dst, src, bytes); });
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
  std::memcpy(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipHostMalloc(void** p, size_t bytes, unsigned) {
  *p = std::aligned_alloc(256, (bytes + 255) & ~size_t(255));
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* p) {
  std::free(p);
  return hipSuccess;
}

namespace lti {

// The classification rules of the kernels (sizes each family covers).
int reduce_class(int n, int m, int p) {
  const int s = (std::max(n + p, n + m) + 15) / 16;
  if (n <= kMaxRegReduceN && s <= kNumRegClasses) return s - 1;
  return n <= kMaxGlobalReduceN ? kReduceGlobal : kReduceBlocked;
}
size_t reduce_work_bytes(int n, int m, int p) { return reduce_class(n, m, p) >= kReduceGlobal ? 4096 : 0; }
size_t reduce_blocked_work_bytes(int, int, int) { return 4096; }
size_t reduce_ht_work_bytes(int, int, int) { return 4096; }
size_t reduced_bytes(int n, int m, int p, bool) {
  return 256 * 13 + 8 * ((size_t)hlen(n) * 2 + (size_t)n * n * 3 + (size_t)vlen(n) + n + (size_t)(n + p) * (m + p) * 4);
}
void reduced_layout(void* base, int n, int m, int p, int trans, ReducedModel* o, bool) {
  std::memset(o, 0, sizeof(*o));
  char* b = static_cast<char*>(base);
  o->D = reinterpret_cast<double*>(b);  // the stand-in kernels use D only
  o->n = n;
  o->m = m;
  o->p = p;
  o->trans = trans;
}
int sweep_class(int precision, int n, int m) {
  if (n < 1 || n > kMaxN || m < 1 || m > kMaxRhs) return -1;
  const int ri = (n <= 64) ? 0 : (n <= 128) ? 1 : 2;
  const int mi = (m <= 1) ? 0 : (m <= 2) ? 1 : (m <= 4) ? 2 : (m <= 8) ? 3 : 4;
  if (ri == 2 && mi == 4) return -1;
  return (precision * kNumRowClasses + ri) * kNumRhsClasses + mi;
}
int sweep16_class(int precision, int n, int mc) {
  if (n < 1 || n > 64 || mc < 1 || mc > 4) return -1;
  const int ri = (n <= 16) ? 0 : (n <= 32) ? 1 : 2;
  const int mi = (mc <= 1) ? 0 : (mc <= 2) ? 1 : 2;
  return (precision * 3 + ri) * 3 + mi;
}
int sweep32_class(int precision, int n, int mc) {
  if (n <= 64 || n > 128 || mc < 1 || mc > 4) return -1;
  const int ri = (n <= 96) ? 0 : 1;
  const int mi = (mc <= 1) ? 0 : (mc <= 2) ? 1 : 2;
  return (precision * 2 + ri) * 3 + mi;
}
int sweep_wg_class(int precision, int n, int mc) {
  if (n <= kMaxN || n > 1024 || mc < 1 || mc > 4) return -1;
  return precision * 3 + ((mc <= 1) ? 0 : (mc <= 2) ? 1 : 2);
}

hipError_t launch_summarize(const FinEntry* tab, PointSummary* out, int n, hipStream_t s) {
  s->push([tab, out, n] {
    for (int i = 0; i < n; ++i) {
      PointSummary ps{};
      for (uint64_t k = 0; k < tab[i].K; ++k) {
        const lti_point_info& pi = tab[i].info[k];
        if (pi.path < 8) ps.count[pi.path]++;
        if (pi.est_rel_err > ps.max_est) ps.max_est = pi.est_rel_err;
      }
      out[i] = ps;
    }
  });
  return hipSuccess;
}

hipError_t launch_zero(const ZeroLaunch& Z, hipStream_t s) {
  s->push([Z] {
    for (int i = 0; i < Z.n; ++i) std::memset(Z.e[i].p, 0, 4 * (size_t)Z.e[i].words);
  });
  return hipSuccess;
}

hipError_t launch_reduce(const ReduceLaunch& L, int, hipStream_t s) {
  s->push([L] {
    for (int i = 0; i < L.njobs; ++i) {
      const ReduceJob& j = L.jobs[i];  // the table was uploaded before, in stream order
      const ModelIn in(j);
      for (int a = 0; a < j.out.p; ++a)
        for (int c = 0; c < j.out.m; ++c) j.out.D[a * j.out.m + c] = in.d(a, c);
    }
  });
  return hipSuccess;
}
hipError_t launch_reduce_blocked(const ReduceJob*, int, hipStream_t) { return hipSuccess; }

static std::mutex g_merge_mu;  // merged point records of the sweep stand-ins

void sweep_stub(const SweepLaunch& L) {
  for (int t = 0; t < L.ntiles; ++t) {
    int s = 0;
    for (int i = 1; i < L.nseg; ++i)
      if (t >= (int)L.seg[i].tile0) s = i;
    const SweepSeg& g = L.seg[s];
    const ReqDesc& rd = g.rd;
    const uint32_t local = g.first + (uint32_t)(t - (int)g.tile0);
    const uint32_t fb = local / g.S, grp = local % g.S;
    const uint32_t start = fb * g.F, count = std::min((uint32_t)g.F, g.K - start);
    const int j0 = (int)grp * g.mc, mc = std::min((int)g.mc, rd.m - j0);
    for (uint32_t f = 0; f < count; ++f) {
      const int64_t k = (int64_t)start + f;
      const int kind = (int)((rd.flags >> 8) & 3u);
      const double w = rd.omega[kind == kPointsS ? 2 * k : k];
      double* G = rd.G + (size_t)k * rd.p * rd.m * 2;
      for (int j = j0; j < j0 + mc; ++j)
        for (int a = 0; a < rd.p; ++a) {
          const int idx = g_index(rd, a, j);
          G[2 * idx] = rd.D[a * rd.m + j] + w * (1.0 + a + 10.0 * j);
          G[2 * idx + 1] = 0.5 * j * w;
        }
      uint32_t* rec = reinterpret_cast<uint32_t*>(rd.info) + 2 * k;
      const uint32_t w1 = (uint32_t)(1 + j0) | (1u << 8);
      if (rd.flags & kFlagMergeInfo) {
        // column groups of one point can be on two streams at once (the
        // device merges with atomic maxima)
        std::lock_guard<std::mutex> lk(g_merge_mu);
        rec[0] = std::max(rec[0], 0u);
        rec[1] = std::max(rec[1], w1);
      } else {
        rec[0] = 0u;
        rec[1] = w1;
      }
    }
  }
}

hipError_t launch_sweep(int, const SweepLaunch& L, size_t, hipStream_t s) {
  s->push([L] { sweep_stub(L); });
  return hipSuccess;
}
hipError_t launch_sweep16(int, const SweepLaunch& L, hipStream_t s) {
  s->push([L] { sweep_stub(L); });
  return hipSuccess;
}
hipError_t launch_sweep32(int, const SweepLaunch& L, hipStream_t s) {
  s->push([L] { sweep_stub(L); });
  return hipSuccess;
}
hipError_t launch_sweep_wg(int, const SweepLaunch& L, hipStream_t s) {
  s->push([L] { sweep_stub(L); });
  return hipSuccess;
}
hipError_t launch_sweep_desc(int, const SweepLaunch& L, hipStream_t s) {
  s->push([L] { sweep_stub(L); });
  return hipSuccess;
}
hipError_t launch_refine_dd(const DDLaunch& L, int grid, hipStream_t s) {
  if (L.nseg <= 0) return hipSuccess;
  if (L.nseg > kMaxDDSegs || grid <= 0) return hipErrorInvalidValue;
  s->push([L] {
    for (int i = 0; i < L.nseg; ++i) {
      if (L.seg[i].rd.fbq[0] != 0u) std::abort();  // the stand-in sweeps queue nothing
    }
  });
  return hipSuccess;
}

}  // namespace lti
