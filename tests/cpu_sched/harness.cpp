// Scheduler harness: the serving runtime (runtime.cpp) driven by several
// client threads against the no-op executor of fake_device.cpp, for
// ThreadSanitizer / AddressSanitizer runs on the CPU.  Exercises admission
// under arena and pinned-staging pressure, model reuse and eviction, the
// pending-queue bound, column splits, the transposed solve, device- and
// host-memory requests, polling with every timeout kind, and destroy with
// requests still outstanding.  Every result is checked against the
// stand-in kernels' formula.  Exit status 0 on success.
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "lti_freqresp.h"

namespace {

std::atomic<int> g_fail{0};

#define CHECK(cond, ...)                          \
  do {                                            \
    if (!(cond)) {                                \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);          \
      std::fprintf(stderr, "\n");                 \
      g_fail++;                                   \
    }                                             \
  } while (0)

struct Req {
  int n, m, p, K, mem, points;
  uint64_t key;
  std::vector<double> A, B, C, D, w, G;
  std::vector<lti_point_info> info;
  uint64_t id = 0;
};

void fill(Req& r, std::mt19937_64& rng) {
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  r.A.resize((size_t)r.n * r.n);
  r.B.resize((size_t)r.n * r.m);
  r.C.resize((size_t)r.p * r.n);
  r.D.resize((size_t)r.p * r.m);
  for (auto* v : {&r.A, &r.B, &r.C, &r.D})
    for (double& x : *v) x = u(rng);
  r.w.resize((size_t)r.K * (r.points == LTI_POINTS_S ? 2 : 1));
  for (double& x : r.w) x = 10.0 * u(rng);
  r.G.assign((size_t)r.K * r.p * r.m * 2, std::nan(""));
  r.info.assign(r.K, lti_point_info{});
}

// G(i, jj) as the stand-in kernels write it (see fake_device.cpp).
void check(const Req& r) {
  const bool trans = r.p < r.m;
  for (int k = 0; k < r.K; ++k) {
    const double w = r.w[(size_t)k * (r.points == LTI_POINTS_S ? 2 : 1)];
    for (int i = 0; i < r.p; ++i)
      for (int jj = 0; jj < r.m; ++jj) {
        // solved system: transposed -> row a = jj, column j = i
        const int a = trans ? jj : i, j = trans ? i : jj;
        const double re = r.D[(size_t)i * r.m + jj] + w * (1.0 + a + 10.0 * j);
        const double im = 0.5 * j * w;
        const double* g = &r.G[((size_t)k * r.p * r.m + (size_t)i * r.m + jj) * 2];
        if (g[0] != re || g[1] != im) {
          CHECK(false, "request n=%d m=%d p=%d K=%d: G[%d][%d][%d] = (%g, %g), want (%g, %g)", r.n, r.m, r.p,
                r.K, k, i, jj, g[0], g[1], re, im);
          return;
        }
      }
    CHECK(r.info[k].path == LTI_PATH_REFINED || r.info[k].path == LTI_PATH_FP64, "path");
  }
}

int submit(lti_ctx* c, Req& r) {
  lti_request q{};
  q.nx = r.n;
  q.nu = r.m;
  q.ny = r.p;
  q.mem = r.mem;
  q.A = r.A.data();
  q.B = r.B.data();
  q.C = r.C.data();
  q.D = r.D.data();
  q.omega = r.w.data();
  q.n_omega = r.K;
  q.precision = LTI_PREC_REFINED;
  q.points = r.points;
  q.model_key = r.key;
  q.G_out = r.G.data();
  q.info_out = r.info.data();
  return lti_freqresp_submit(c, &q, &r.id);
}

void client(lti_ctx* c, int tid, int nreq) {
  std::mt19937_64 rng(1234 + tid);
  std::vector<Req> reqs(nreq);
  std::vector<int> pending;
  for (int i = 0; i < nreq; ++i) {
    Req& r = reqs[i];
    r.n = 1 + (int)(rng() % 300);
    if (rng() % 16 == 0) r.n = 257 + (int)(rng() % 700);
    r.m = 1 + (int)(rng() % 8);
    r.p = 1 + (int)(rng() % 8);
    r.K = 1 + (int)(rng() % 1500);
    r.mem = (rng() % 3 == 0) ? LTI_MEM_DEVICE : LTI_MEM_HOST;  // "device" = host memory here
    r.points = (int)(rng() % 3);
    r.key = (rng() % 4 == 0) ? 1 + rng() % 5 : 0;
    if (r.key) {  // keyed models: fixed sizes per key, so reuse happens
      r.n = 20 + 10 * (int)r.key;
      r.m = 3;
      r.p = 2 + (int)(r.key % 3);
    }
    fill(r, rng);
    if (r.key) {  // same key, same content
      std::mt19937_64 krng(99 + r.key);
      std::uniform_real_distribution<double> u(-1.0, 1.0);
      for (auto* v : {&r.A, &r.B, &r.C, &r.D})
        for (double& x : *v) x = u(krng);
    }
    for (;;) {
      const int rc = submit(c, r);
      if (rc == LTI_OK) break;
      CHECK(rc == LTI_EAGAIN, "submit rc %d", rc);
      if (rc != LTI_EAGAIN) return;
      // queue full: collect one of ours and retry
      if (!pending.empty()) {
        Req& o = reqs[pending.front()];
        lti_result res{};
        const int prc = lti_freqresp_poll(c, o.id, -1, &res);
        CHECK(prc == LTI_OK, "poll rc %d", prc);
        check(o);
        pending.erase(pending.begin());
      } else {
        std::this_thread::sleep_for(std::chrono::microseconds(100));
      }
    }
    pending.push_back(i);
    // poll some with short timeouts, some not at all yet
    if (rng() % 3 == 0 && !pending.empty()) {
      Req& o = reqs[pending.front()];
      lti_result res{};
      const int prc = lti_freqresp_poll(c, o.id, (int)(rng() % 2) * 200, &res);
      if (prc == LTI_OK) {
        CHECK(res.n_points == o.K, "n_points");
        CHECK(res.n_refined == o.K, "n_refined %lld of %d", (long long)res.n_refined, o.K);
        check(o);
        pending.erase(pending.begin());
      } else {
        CHECK(prc == LTI_PENDING, "poll rc %d", prc);
      }
    }
  }
  for (int idx : pending) {
    lti_result res{};
    const int prc = lti_freqresp_poll(c, reqs[idx].id, -1, &res);
    CHECK(prc == LTI_OK, "final poll rc %d", prc);
    check(reqs[idx]);
  }
}

}  // namespace

int main(int argc, char** argv) {
  const int nthreads = argc > 1 ? std::atoi(argv[1]) : 4;
  const int nreq = argc > 2 ? std::atoi(argv[2]) : 60;
  const size_t arena_bytes = size_t(48) << 20;
  void* arena = std::aligned_alloc(256, arena_bytes);
  lti_config cfg{};
  cfg.abi_version = LTI_ABI_VERSION;
  cfg.arena = arena;
  cfg.arena_bytes = arena_bytes;
  cfg.max_pending = 24;
  cfg.max_batch_tiles = 2048;
  cfg.host_staging_bytes = size_t(8) << 20;  // small: requests wait for pinned staging too
  cfg.flags = LTI_CFG_KERNEL_TIMING;
  lti_ctx* c = nullptr;
  int rc = lti_freqresp_create(&cfg, &c);
  CHECK(rc == LTI_OK, "create rc %d", rc);
  if (!c) return 1;
  std::vector<std::thread> th;
  for (int t = 0; t < nthreads; ++t) th.emplace_back(client, c, t, nreq);
  for (auto& t : th) t.join();
  lti_stats st{};
  lti_freqresp_stats(c, &st);
  CHECK(st.requests_done == st.requests_submitted, "done %llu of %llu", (unsigned long long)st.requests_done,
        (unsigned long long)st.requests_submitted);
  CHECK(st.arena_peak_bytes <= arena_bytes, "arena peak");
  CHECK(st.reduction_cache_hits > 0, "no model reuse happened");
  // errors: a request that can never fit, an unknown id
  {
    Req big;
    big.n = 8; big.m = 16; big.p = 16; big.K = 200000; big.mem = LTI_MEM_HOST; big.points = 0; big.key = 0;
    std::mt19937_64 rng(5);
    fill(big, rng);
    CHECK(submit(c, big) == LTI_ENOSPC, "ENOSPC");
    lti_result res{};
    CHECK(lti_freqresp_poll(c, 987654321ull, 0, &res) == LTI_ENOENT, "ENOENT");
  }
  // destroy with requests still outstanding (never collected)
  std::vector<Req> left(6);
  std::mt19937_64 rng(77);
  for (Req& r : left) {
    r.n = 40; r.m = 2; r.p = 3; r.K = 700; r.mem = LTI_MEM_HOST; r.points = 0; r.key = 0;
    fill(r, rng);
    CHECK(submit(c, r) == LTI_OK, "late submit");
  }
  CHECK(lti_freqresp_destroy(c) == LTI_OK, "destroy");
  std::free(arena);
  if (g_fail) {
    std::fprintf(stderr, "%d failures\n", g_fail.load());
    return 1;
  }
  std::printf("scheduler harness: %d threads x %d requests ok (reductions %llu, reuse %llu, batches %llu)\n",
              nthreads, nreq, (unsigned long long)st.reductions, (unsigned long long)st.reduction_cache_hits,
              (unsigned long long)st.sweep_launches);
  return 0;
}
