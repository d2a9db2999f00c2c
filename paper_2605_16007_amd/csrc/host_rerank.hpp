// Exact re-rank on host cores (Sec. 3.3.4) for indexes whose raw vectors stay
// in pinned host memory: a persistent thread pool and the per-query kernel.
#pragma once
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

namespace rbq {

class ThreadPool {
 public:
  explicit ThreadPool(int threads);
  ~ThreadPool();
  ThreadPool(const ThreadPool&) = delete;
  ThreadPool& operator=(const ThreadPool&) = delete;
  void submit(std::function<void()> task);
  int size() const { return (int)workers_.size(); }

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  std::deque<std::function<void()>> tasks_;
  bool stop_ = false;
  std::vector<std::thread> workers_;
};

// Counts outstanding tasks; wait() returns when all have called done().
class Latch {
 public:
  void add(int64_t n);
  void done();
  void wait();

 private:
  std::mutex mu_;
  std::condition_variable cv_;
  int64_t n_ = 0;
};

// Queries [q0, q1) of a batch: for each, the exact squared L2 distance (FP64
// accumulation over the FP32 inputs) to each of its candidates (64-bit keys
// whose low word is the vector id; KEY_NONE slots are skipped), then the best
// k(i) by (distance, id), written as FP32 with (-1, +inf) padding up to
// k_stride. X is n x d host rows; q rows have stride d; cand rows stride R.
void host_rerank_rows(const float* X, int64_t n, int d, const float* q, const uint64_t* cand, int R,
                      const int32_t* rowk, int k_stride, int64_t q0, int64_t q1, int64_t* ids,
                      float* dist);

}  // namespace rbq
