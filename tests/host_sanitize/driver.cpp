// Thread-sanitizer driver of the serving loop and the host re-rank pool:
// several submitting threads against a multi-lane server (admission by
// workspace, batching, result publication, polling and waiting), a replay
// with its collector thread, destroy with requests in flight, and the host
// re-rank's thread pool and latch under concurrent submitters.
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "host_rerank.hpp"
#include "server.hpp"

using namespace rbq;

static int failures = 0;
#define EXPECT(c)                                                     \
  do {                                                                \
    if (!(c)) {                                                       \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static void serve(rbq_index* idx) {
  rbq_server_params p;
  server_params_default(&p);
  p.lanes = 3;
  p.max_batch = 16;
  p.queue_cap = 64;
  p.max_nprobe = 32;
  p.max_k = 20;
  p.max_rerank = 40;
  p.mem_budget = 1 << 20;  // small enough that admission cuts batches
  rbq_server* srv = server_create(idx, p);
  std::vector<std::thread> th;
  std::atomic<int> done{0};
  for (int t = 0; t < 4; ++t)
    th.emplace_back([&, t] {
      std::vector<float> q(idx->d);
      int64_t ids[20];
      float dist[20];
      for (int r = 0; r < 300; ++r) {
        const int k = 1 + (r * 7 + t) % 20;
        q[0] = (float)(t * 1000 + r);
        uint64_t ticket = 0;
        rbq_status st;
        while ((st = server_submit(srv, q.data(), 1 + r % 32, k, std::max(k, 1 + (r * 3) % 40), &ticket)) ==
               RBQ_EAGAIN)
          std::this_thread::yield();
        EXPECT(st == RBQ_OK);
        int64_t tdone = 0, lat = 0;
        const int got = (r % 2) ? server_collect(srv, ticket, ids, dist, -1, &tdone, &lat)
                                : [&] {
                                    int g = 0;
                                    while (!(g = server_collect(srv, ticket, ids, dist, 0, &tdone, &lat)))
                                      std::this_thread::yield();
                                    return g;
                                  }();
        EXPECT(got == 1);
        for (int c = 0; c < k; ++c) EXPECT(ids[c] == (int64_t)(t * 1000 + r) * 1000 + c);
        ++done;
      }
    });
  for (auto& x : th) x.join();
  EXPECT(done.load() == 1200);
  rbq_server_stats st;
  server_stats(srv, &st);
  EXPECT(st.completed == 1200);
  // a replay (submitter and collector threads inside the library)
  const int n = 200;
  std::vector<float> qs((size_t)n * idx->d, 0.f);
  std::vector<int32_t> np(n), kk(n), rr(n);
  std::vector<double> arr(n);
  std::vector<int64_t> rid((size_t)n * 20);
  std::vector<float> rdist((size_t)n * 20);
  std::vector<double> lat(n);
  for (int i = 0; i < n; ++i) {
    qs[(size_t)i * idx->d] = (float)i;
    np[i] = 1 + i % 32;
    kk[i] = 1 + i % 20;
    rr[i] = 40;
    arr[i] = 1e-5 * i;
  }
  rbq_replay_io io{};
  io.q = qs.data();
  io.nprobe = np.data();
  io.k = kk.data();
  io.rerank_n = rr.data();
  io.arrival_s = arr.data();
  io.ids = rid.data();
  io.sqdist = rdist.data();
  io.latency_s = lat.data();
  io.n = n;
  io.k_stride = 20;
  server_replay(srv, io);
  for (int i = 0; i < n; ++i) EXPECT(rid[(size_t)i * 20] == (int64_t)i * 1000);
  // destroy with requests still queued
  for (int r = 0; r < 40; ++r) {
    uint64_t ticket;
    std::vector<float> q(idx->d, 1.f);
    if (server_submit(srv, q.data(), 4, 4, 4, &ticket) != RBQ_OK) break;
  }
  server_destroy(srv);
}

static void rerank_pool() {
  const int n = 512, d = 8, R = 16, nq = 64;
  std::vector<float> X((size_t)n * d), Q((size_t)nq * d);
  for (size_t i = 0; i < X.size(); ++i) X[i] = (float)((i * 37) % 101);
  for (size_t i = 0; i < Q.size(); ++i) Q[i] = (float)((i * 13) % 97);
  std::vector<uint64_t> cand((size_t)nq * R);
  for (int i = 0; i < nq; ++i)
    for (int r = 0; r < R; ++r) cand[(size_t)i * R + r] = (uint64_t)((i * 5 + r * 31) % n);
  // the reference, computed on this thread before any other starts
  std::vector<int64_t> ids((size_t)nq * 4);
  std::vector<float> dist((size_t)nq * 4);
  host_rerank_rows(X.data(), n, d, Q.data(), cand.data(), R, nullptr, 4, 0, nq, ids.data(), dist.data());
  ThreadPool pool(6);
  std::vector<std::thread> subs;
  for (int s = 0; s < 3; ++s)
    subs.emplace_back([&, s] {
      for (int it = 0; it < 20; ++it) {
        Latch latch;
        std::vector<int64_t> li((size_t)nq * 4);
        std::vector<float> ld((size_t)nq * 4);
        for (int q0 = 0; q0 < nq; q0 += 8) {
          latch.add(1);
          pool.submit([&, q0] {
            host_rerank_rows(X.data(), n, d, Q.data(), cand.data(), R, nullptr, 4, q0, q0 + 8, li.data(),
                             ld.data());
            latch.done();
          });
        }
        latch.wait();
        EXPECT(li == ids);
        EXPECT(ld == dist);
      }
    });
  for (auto& x : subs) x.join();
}

int main() {
  rbq_index idx;
  idx.d = 8;
  idx.ld = 8;
  idx.nlist = 64;
  idx.n = 4096;
  idx.max_list_len = 128;
  serve(&idx);
  rerank_pool();
  std::printf("host sanitize driver: %d failures\n", failures);
  return failures ? 1 : 0;
}
