// Serving loop: continuous batching of single-query requests over a resident
// index (lanes = host threads with their own stream and fixed workspace).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "index.hpp"

namespace rbq {

enum class ReqState : uint8_t { Free, Waiting, Running, Done, Failed };

struct Request {
  uint32_t gen = 0;  // bumped on every reuse of the slot; part of the ticket
  ReqState state = ReqState::Free;
  int32_t nprobe = 0, k = 0, R = 0;
  int64_t t_submit = 0, t_done = 0;  // steady-clock ns
  rbq_status err = RBQ_OK;
  std::string msg;
};

struct Lane {
  hipStream_t stream = nullptr;
  char* ws = nullptr;      // device workspace, mem_budget bytes
  float* dq = nullptr;     // device queries, max_batch x d
  int64_t* dids = nullptr; // device results, max_batch x max_k
  float* ddist = nullptr;
  float* hq = nullptr;     // pinned staging
  int32_t* hspec = nullptr;
  int64_t* hids = nullptr;
  float* hdist = nullptr;
  std::thread thread;
};

}  // namespace rbq

struct rbq_server {
  rbq_index* idx = nullptr;
  rbq_server_params p{};
  int d = 0;

  std::mutex mu;                      // requests, pending, stats
  std::condition_variable cv_work;    // lanes: work arrived or stop
  std::condition_variable cv_done;    // waiters: a request finished or a slot freed
  std::mutex admit_mu;                // one lane forms a batch at a time
  std::vector<rbq::Request> req;      // queue_cap slots
  std::vector<float> qbuf;            // queue_cap x d submitted queries
  std::vector<int64_t> rids;          // queue_cap x max_k results
  std::vector<float> rdist;
  std::vector<uint32_t> free_slots;
  std::deque<uint32_t> pending;       // waiting requests, arrival order
  bool stop = false;
  rbq_server_stats stats{};
  std::vector<rbq::Lane> lanes;

  ~rbq_server();
};

namespace rbq {

int64_t now_ns();
void server_params_default(rbq_server_params* p);
rbq_server* server_create(rbq_index* idx, const rbq_server_params& p);
void server_destroy(rbq_server* s);
// returns RBQ_OK / RBQ_EAGAIN / RBQ_ENOMEM via exceptions for errors
rbq_status server_submit(rbq_server* s, const float* q, int nprobe, int k, int R, uint64_t* ticket);
// done: 0 not finished; 1 finished (outputs written, slot released). Throws
// the batch's error for a failed request (slot released).
int server_collect(rbq_server* s, uint64_t ticket, int64_t* ids, float* dist, int64_t timeout_us,
                   int64_t* t_done_ns, int64_t* latency_ns);
void server_stats(rbq_server* s, rbq_server_stats* st);
void server_replay(rbq_server* s, const rbq_replay_io& io);
void replay_plain(rbq_index* idx, const rbq_replay_io& io);

}  // namespace rbq
