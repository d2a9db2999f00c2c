// Serving loop: continuous batching over a resident index.
//
// Requests arrive one query at a time (rbq_submit) and wait in arrival order.
// Each lane is a host thread with its own HIP stream, a device workspace of
// mem_budget bytes and pinned staging buffers. A free lane forms the next
// batch from the oldest waiting requests, as many as fit max_batch and whose
// joint workspace need (a function of the batch size, the widest nprobe, the
// largest k and rerank_n and the number of (query, list) pairs) fits
// mem_budget, then runs them as one mixed batch, so that requests that
// arrived while other batches were on the device are admitted as soon as a
// lane and memory free up, and several batches' kernels overlap on the device.
#include "server.hpp"

#include <algorithm>
#include <chrono>
#include <cstring>

namespace rbq {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

void server_params_default(rbq_server_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->lanes = 2;
  p->max_batch = 1024;
  p->queue_cap = 65536;
  p->max_nprobe = 0;  // min(nlist, 256)
  p->max_k = 100;
  p->max_rerank = 1000;
  p->mem_budget = (int64_t)1 << 30;
}

namespace {

constexpr uint32_t kSlotBits = 32;

uint64_t make_ticket(uint32_t gen, uint32_t slot) { return ((uint64_t)gen << kSlotBits) | slot; }

// Minimal candidate-row budget of a batch: one chunk of probe ranks (the
// running top-R plus a pool of R keys per query).
int64_t min_pool(int64_t nb, int R) { return 2 * nb * (int64_t)R * 8; }

size_t batch_need(const rbq_index* idx, int64_t nb, int np, int k, int R, int64_t pairs) {
  return search_workspace_bytes(idx, nb, np, k, R, pairs, min_pool(nb, R));
}

struct Snapshot {
  std::vector<int32_t> np, k, R;  // prefix maxima over the waiting requests
  std::vector<int64_t> pairs;     // prefix sums of nprobe
};

// The most requests from the front of the snapshot whose batch fits the
// workspace (the need grows with every prefix, so a binary search suffices).
int admit_count(const rbq_server* S, const Snapshot& sn) {
  const int m = (int)sn.np.size();
  int lo = 1, hi = m;  // a single request always fits (checked at create)
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    const size_t need = batch_need(S->idx, mid, sn.np[mid - 1], sn.k[mid - 1], sn.R[mid - 1],
                                   sn.pairs[mid - 1]);
    if (need <= (size_t)S->p.mem_budget)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

void run_batch(rbq_server* S, Lane& L, const std::vector<uint32_t>& batch) {
  const int nb = (int)batch.size();
  const int d = S->d;
  int np = 0, k = 0, R = 0;
  int64_t pairs = 0;
  for (int t = 0; t < nb; ++t) {
    const Request& r = S->req[batch[t]];
    std::memcpy(L.hq + (size_t)t * d, &S->qbuf[(size_t)batch[t] * d], (size_t)d * sizeof(float));
    L.hspec[t] = r.nprobe;
    L.hspec[nb + t] = r.k;
    L.hspec[2 * nb + t] = r.R;
    np = std::max(np, r.nprobe);
    k = std::max(k, r.k);
    R = std::max(R, r.R);
    pairs += r.nprobe;
  }
  RBQ_HIP(hipMemcpyAsync(L.dq, L.hq, (size_t)nb * d * sizeof(float), hipMemcpyHostToDevice, L.stream));
  SearchIO io;
  io.q_nprobe = L.hspec;
  io.q_k = L.hspec + nb;
  io.q_R = L.hspec + 2 * nb;
  io.ws_base = L.ws;
  io.ws_cap = (size_t)S->p.mem_budget;
  // the candidate rows get the largest budget whose whole workspace (sized by
  // the plan at that budget) still fits mem_budget; admission checked that the
  // smallest one does
  io.pool_budget = std::max<int64_t>(
      min_pool(nb, R),
      fit_pool_budget(S->idx, nb, np, k, R, pairs, (size_t)S->p.mem_budget, min_pool(nb, R)));
  search(S->idx, L.dq, nb, np, k, R, L.dids, L.ddist, L.stream, io);
  RBQ_HIP(hipMemcpyAsync(L.hids, L.dids, (size_t)nb * k * sizeof(int64_t), hipMemcpyDeviceToHost,
                         L.stream));
  RBQ_HIP(hipMemcpyAsync(L.hdist, L.ddist, (size_t)nb * k * sizeof(float), hipMemcpyDeviceToHost,
                         L.stream));
  RBQ_HIP(hipStreamSynchronize(L.stream));
  const int64_t t_done = now_ns();
  const int mk = S->p.max_k;
  for (int t = 0; t < nb; ++t) {  // the slots are this lane's until marked done
    const uint32_t slot = batch[t];
    const int kr = S->req[slot].k;
    std::memcpy(&S->rids[(size_t)slot * mk], L.hids + (size_t)t * k, kr * sizeof(int64_t));
    std::memcpy(&S->rdist[(size_t)slot * mk], L.hdist + (size_t)t * k, kr * sizeof(float));
  }
  std::lock_guard<std::mutex> g(S->mu);
  for (uint32_t slot : batch) {
    S->req[slot].state = ReqState::Done;
    S->req[slot].t_done = t_done;
  }
  S->stats.completed += nb;
}

void lane_main(rbq_server* S, int li) {
  Lane& L = S->lanes[li];
  (void)hipSetDevice(S->idx->device);
  const int maxb = S->p.max_batch;
  std::vector<uint32_t> batch;
  batch.reserve(maxb);
  Snapshot sn;
  for (;;) {
    batch.clear();
    {
      std::unique_lock<std::mutex> al(S->admit_mu);
      int m = 0;
      {
        std::unique_lock<std::mutex> lk(S->mu);
        S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty(); });
        if (S->pending.empty()) return;  // stopping, and nothing is left
        m = (int)std::min<size_t>(S->pending.size(), (size_t)maxb);
        sn.np.resize(m);
        sn.k.resize(m);
        sn.R.resize(m);
        sn.pairs.resize(m);
        int a = 0, b = 0, c = 0;
        int64_t pr = 0;
        for (int t = 0; t < m; ++t) {
          const Request& r = S->req[S->pending[t]];
          a = std::max(a, r.nprobe);
          b = std::max(b, r.k);
          c = std::max(c, r.R);
          pr += r.nprobe;
          sn.np[t] = a;
          sn.k[t] = b;
          sn.R[t] = c;
          sn.pairs[t] = pr;
        }
      }
      // (only lanes pop from `pending`, and only under admit_mu, so its front
      // m entries are unchanged while the lock is dropped)
      const int c = admit_count(S, sn);
      std::lock_guard<std::mutex> lk(S->mu);
      for (int t = 0; t < c; ++t) {
        const uint32_t slot = S->pending.front();
        S->pending.pop_front();
        S->req[slot].state = ReqState::Running;
        batch.push_back(slot);
      }
      S->stats.batches += 1;
      S->stats.max_batch_seen = std::max<int64_t>(S->stats.max_batch_seen, c);
      if (c < m) S->stats.budget_cuts += 1;
      if (!S->pending.empty()) S->cv_work.notify_one();
    }
    rbq_status err = RBQ_OK;
    std::string msg;
    try {
      run_batch(S, L, batch);
    } catch (const Error& e) {
      err = e.status;
      msg = e.what();
    } catch (const std::bad_alloc&) {
      err = RBQ_ENOMEM;
      msg = "host allocation failed";
    } catch (const std::exception& e) {
      err = RBQ_EDEVICE;
      msg = e.what();
    }
    if (err != RBQ_OK) {
      (void)hipStreamSynchronize(L.stream);  // nothing of the batch may still use the workspace
      (void)hipGetLastError();
      std::lock_guard<std::mutex> g(S->mu);
      for (uint32_t slot : batch) {
        S->req[slot].state = ReqState::Failed;
        S->req[slot].err = err;
        S->req[slot].msg = msg;
        S->req[slot].t_done = now_ns();
      }
      S->stats.completed += (int64_t)batch.size();
    }
    S->cv_done.notify_all();
  }
}

}  // namespace

rbq_server* server_create(rbq_index* idx, const rbq_server_params& p0) {
  rbq_server_params p = p0;
  if (p.max_nprobe == 0) p.max_nprobe = std::min(idx->nlist, 256);
  RBQ_CHECK(p.lanes >= 1 && p.lanes <= 8, "lanes must be in [1, 8]");
  RBQ_CHECK(p.max_batch >= 1 && p.max_batch <= 65536, "max_batch must be in [1, 65536]");
  RBQ_CHECK(p.queue_cap >= 1 && p.queue_cap <= (1 << 22), "queue_cap must be in [1, 2^22]");
  RBQ_CHECK(p.max_nprobe >= 1 && p.max_nprobe <= std::min(idx->nlist, MAX_SEL),
            "max_nprobe must be in [1, min(nlist, 4096)]");
  RBQ_CHECK(p.max_rerank >= 1 && p.max_rerank <= MAX_R, "max_rerank must be in [1, 3840]");
  RBQ_CHECK(p.max_k >= 1 && p.max_k <= p.max_rerank, "max_k must be in [1, max_rerank]");
  RBQ_CHECK(p.mem_budget >= ((int64_t)1 << 20), "mem_budget must be at least 1 MiB");
  for (int32_t r : p.reserved) RBQ_CHECK(r == 0, "reserved fields must be zero");
  RBQ_CHECK(batch_need(idx, 1, p.max_nprobe, p.max_k, p.max_rerank, p.max_nprobe) <=
                (size_t)p.mem_budget,
            "mem_budget is too small for a single request at the server's limits");
  RBQ_CHECK((int64_t)p.max_batch * p.max_nprobe <= (int64_t)INT32_MAX, "max_batch * max_nprobe too large");

  std::unique_ptr<rbq_server> S(new rbq_server());
  S->idx = idx;
  S->p = p;
  S->d = idx->d;
  S->req.resize(p.queue_cap);
  S->qbuf.resize((size_t)p.queue_cap * idx->d);
  S->rids.resize((size_t)p.queue_cap * p.max_k);
  S->rdist.resize((size_t)p.queue_cap * p.max_k);
  S->free_slots.reserve(p.queue_cap);
  for (int i = p.queue_cap - 1; i >= 0; --i) S->free_slots.push_back((uint32_t)i);

  RBQ_HIP(hipSetDevice(idx->device));
  S->lanes.resize(p.lanes);
  const size_t mb = (size_t)p.max_batch;
  auto dev_alloc = [](void** ptr, size_t bytes) {
    if (hipMalloc(ptr, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      throw Error(RBQ_ENOMEM, "device allocation for the server failed");
    }
  };
  auto host_alloc = [](void** ptr, size_t bytes) {
    if (hipHostMalloc(ptr, bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      *ptr = nullptr;
      throw Error(RBQ_ENOMEM, "pinned host allocation for the server failed");
    }
  };
  for (auto& L : S->lanes) {
    RBQ_HIP(hipStreamCreateWithFlags(&L.stream, hipStreamNonBlocking));
    dev_alloc((void**)&L.ws, (size_t)p.mem_budget);
    dev_alloc((void**)&L.dq, mb * idx->d * sizeof(float));
    dev_alloc((void**)&L.dids, mb * p.max_k * sizeof(int64_t));
    dev_alloc((void**)&L.ddist, mb * p.max_k * sizeof(float));
    host_alloc((void**)&L.hq, mb * idx->d * sizeof(float));
    host_alloc((void**)&L.hspec, mb * 3 * sizeof(int32_t));
    host_alloc((void**)&L.hids, mb * p.max_k * sizeof(int64_t));
    host_alloc((void**)&L.hdist, mb * p.max_k * sizeof(float));
  }
  rbq_server* raw = S.get();
  for (int li = 0; li < p.lanes; ++li) S->lanes[li].thread = std::thread(lane_main, raw, li);
  return S.release();
}

void server_destroy(rbq_server* s) { delete s; }

rbq_status server_submit(rbq_server* S, const float* q, int nprobe, int k, int R, uint64_t* ticket) {
  RBQ_CHECK(q != nullptr && ticket != nullptr, "query or ticket is NULL");
  RBQ_CHECK(nprobe >= 1 && nprobe <= S->p.max_nprobe, "nprobe outside [1, max_nprobe]");
  RBQ_CHECK(R >= 1 && R <= S->p.max_rerank, "rerank_n outside [1, max_rerank]");
  RBQ_CHECK(k >= 1 && k <= S->p.max_k && k <= R, "k outside [1, min(max_k, rerank_n)]");
  RBQ_CHECK(!is_device_ptr(q), "the query must be in host memory");
  {
    std::lock_guard<std::mutex> g(S->mu);
    if (S->stop) throw Error(RBQ_ESTATE, "server is stopping");
    if (S->free_slots.empty()) {
      S->stats.rejected += 1;
      return RBQ_EAGAIN;
    }
    const uint32_t slot = S->free_slots.back();
    S->free_slots.pop_back();
    Request& r = S->req[slot];
    r.state = ReqState::Waiting;
    r.nprobe = nprobe;
    r.k = k;
    r.R = R;
    r.err = RBQ_OK;
    r.msg.clear();
    r.t_submit = now_ns();
    r.t_done = 0;
    std::memcpy(&S->qbuf[(size_t)slot * S->d], q, (size_t)S->d * sizeof(float));
    S->pending.push_back(slot);
    S->stats.submitted += 1;
    *ticket = make_ticket(r.gen, slot);
  }
  S->cv_work.notify_one();
  return RBQ_OK;
}

int server_collect(rbq_server* S, uint64_t ticket, int64_t* ids, float* dist, int64_t timeout_us,
                   int64_t* t_done_ns, int64_t* latency_ns) {
  const uint32_t slot = (uint32_t)(ticket & 0xFFFFFFFFu);
  const uint32_t gen = (uint32_t)(ticket >> kSlotBits);
  std::unique_lock<std::mutex> lk(S->mu);
  auto valid = [&] {
    return slot < S->req.size() && S->req[slot].gen == gen && S->req[slot].state != ReqState::Free;
  };
  RBQ_CHECK(valid(), "unknown or already collected ticket");
  auto finished = [&] {
    const ReqState st = S->req[slot].state;
    return st == ReqState::Done || st == ReqState::Failed;
  };
  if (!finished()) {
    if (timeout_us == 0) return 0;
    if (timeout_us < 0)
      S->cv_done.wait(lk, finished);
    else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), finished))
      return 0;
  }
  Request& r = S->req[slot];
  const rbq_status err = r.err;
  const std::string msg = r.msg;
  if (t_done_ns) *t_done_ns = r.t_done;
  if (latency_ns) *latency_ns = r.t_done - r.t_submit;
  if (r.state == ReqState::Done) {
    if (ids) std::memcpy(ids, &S->rids[(size_t)slot * S->p.max_k], r.k * sizeof(int64_t));
    if (dist) std::memcpy(dist, &S->rdist[(size_t)slot * S->p.max_k], r.k * sizeof(float));
  }
  r.state = ReqState::Free;
  r.gen += 1;
  S->free_slots.push_back(slot);
  lk.unlock();
  S->cv_done.notify_all();  // a submitter may wait for a free slot
  if (err != RBQ_OK) throw Error(err, msg);
  return 1;
}

void server_stats(rbq_server* S, rbq_server_stats* st) {
  std::lock_guard<std::mutex> g(S->mu);
  *st = S->stats;
}

namespace {

void check_replay(const rbq_replay_io& io, int max_k) {
  RBQ_CHECK(io.n >= 0, "n must be >= 0");
  RBQ_CHECK(io.reserved == 0, "reserved must be zero");
  if (io.n == 0) return;
  RBQ_CHECK(io.q && io.nprobe && io.k && io.rerank_n && io.arrival_s && io.ids && io.sqdist &&
                io.latency_s,
            "replay arrays are NULL");
  RBQ_CHECK(io.k_stride >= 1 && io.k_stride <= max_k, "k_stride out of range");
  for (int64_t i = 0; i < io.n; ++i) {
    RBQ_CHECK(io.k[i] >= 1 && io.k[i] <= io.k_stride, "k[i] must be in [1, k_stride]");
    RBQ_CHECK(i == 0 || io.arrival_s[i] >= io.arrival_s[i - 1], "arrival times must not decrease");
  }
}

void pad_row(const rbq_replay_io& io, int64_t i) {
  for (int c = io.k[i]; c < io.k_stride; ++c) {
    io.ids[i * io.k_stride + c] = -1;
    io.sqdist[i * io.k_stride + c] = INFINITY;
  }
}

// Waits until steady-clock time `t` (sleeps while far, then spins).
void wait_until(int64_t t) {
  for (;;) {
    const int64_t now = now_ns();
    if (now >= t) return;
    if (t - now > 200000)
      std::this_thread::sleep_for(std::chrono::nanoseconds(t - now - 100000));
    else
      std::this_thread::yield();
  }
}

}  // namespace

void server_replay(rbq_server* S, const rbq_replay_io& io) {
  check_replay(io, S->p.max_k);
  if (io.n == 0) return;
  const int d = S->d;
  std::vector<uint64_t> tickets(io.n);
  std::mutex rmu;
  std::condition_variable rcv;
  int64_t submitted = 0;     // guarded by rmu
  bool failed = false;       // guarded by rmu
  rbq_status ferr = RBQ_OK;
  std::string fmsg;
  const int64_t t0 = now_ns() + 1000000;
  auto fail = [&](rbq_status e, const std::string& m) {
    std::lock_guard<std::mutex> g(rmu);
    if (!failed) {
      failed = true;
      ferr = e;
      fmsg = m;
    }
    rcv.notify_all();
  };
  std::thread collector([&] {
    try {
      for (int64_t i = 0; i < io.n; ++i) {
        {
          std::unique_lock<std::mutex> lk(rmu);
          rcv.wait(lk, [&] { return submitted > i || failed; });
          if (submitted <= i) return;
        }
        int64_t t_done = 0;
        server_collect(S, tickets[i], io.ids + i * io.k_stride, io.sqdist + i * io.k_stride, -1,
                       &t_done, nullptr);
        pad_row(io, i);
        io.latency_s[i] = (double)(t_done - t0) * 1e-9 - io.arrival_s[i];
      }
    } catch (const Error& e) {
      fail(e.status, e.what());
    } catch (const std::exception& e) {
      fail(RBQ_EDEVICE, e.what());
    }
  });
  try {
    for (int64_t i = 0; i < io.n; ++i) {
      wait_until(t0 + (int64_t)(io.arrival_s[i] * 1e9));
      uint64_t t = 0;
      for (;;) {
        {
          std::lock_guard<std::mutex> g(rmu);
          if (failed) break;
        }
        const rbq_status st = server_submit(S, io.q + (size_t)i * d, io.nprobe[i], io.k[i],
                                            io.rerank_n[i], &t);
        if (st == RBQ_OK) break;
        std::unique_lock<std::mutex> lk(S->mu);  // queue full: wait for a collected slot
        S->cv_done.wait_for(lk, std::chrono::microseconds(200),
                            [&] { return !S->free_slots.empty(); });
      }
      std::lock_guard<std::mutex> g(rmu);
      if (failed) break;
      tickets[i] = t;
      submitted = i + 1;
      rcv.notify_all();
    }
  } catch (const Error& e) {
    fail(e.status, e.what());
  } catch (const std::exception& e) {
    fail(RBQ_EDEVICE, e.what());
  }
  collector.join();
  if (failed) throw Error(ferr, fmsg);
}

void replay_plain(rbq_index* idx, const rbq_replay_io& io) {
  check_replay(io, MAX_R);
  if (io.n == 0) return;
  RBQ_HIP(hipSetDevice(idx->device));
  hipStream_t s = nullptr;
  RBQ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  const int d = idx->d;
  try {
    const int64_t t0 = now_ns() + 1000000;
    for (int64_t i = 0; i < io.n; ++i) {
      RBQ_CHECK(io.nprobe[i] >= 1 && io.nprobe[i] <= std::min(idx->nlist, MAX_SEL), "nprobe[i] out of range");
      RBQ_CHECK(io.rerank_n[i] >= io.k[i] && io.rerank_n[i] <= MAX_R, "rerank_n[i] out of range");
      wait_until(t0 + (int64_t)(io.arrival_s[i] * 1e9));
      search(idx, io.q + (size_t)i * d, 1, io.nprobe[i], io.k[i], io.rerank_n[i],
             io.ids + i * io.k_stride, io.sqdist + i * io.k_stride, s, SearchIO{});
      io.latency_s[i] = (double)(now_ns() - t0) * 1e-9 - io.arrival_s[i];
      pad_row(io, i);
    }
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
    throw;
  }
  RBQ_HIP(hipStreamDestroy(s));
}

}  // namespace rbq

rbq_server::~rbq_server() {
  {
    std::lock_guard<std::mutex> g(mu);
    stop = true;
  }
  cv_work.notify_all();
  for (auto& L : lanes)
    if (L.thread.joinable()) L.thread.join();
  for (auto& L : lanes) {
    if (L.stream) (void)hipStreamSynchronize(L.stream);
    if (L.ws) (void)hipFree(L.ws);
    if (L.dq) (void)hipFree(L.dq);
    if (L.dids) (void)hipFree(L.dids);
    if (L.ddist) (void)hipFree(L.ddist);
    if (L.hq) (void)hipHostFree(L.hq);
    if (L.hspec) (void)hipHostFree(L.hspec);
    if (L.hids) (void)hipHostFree(L.hids);
    if (L.hdist) (void)hipHostFree(L.hdist);
    if (L.stream) (void)hipStreamDestroy(L.stream);
  }
}
