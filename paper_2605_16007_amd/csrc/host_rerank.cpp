#include "host_rerank.hpp"

#include <algorithm>
#include <cmath>
#include <utility>

#include "common.hpp"

namespace rbq {

ThreadPool::ThreadPool(int threads) {
  threads = std::max(1, threads);
  workers_.reserve(threads);
  for (int t = 0; t < threads; ++t)
    workers_.emplace_back([this] {
      for (;;) {
        std::function<void()> task;
        {
          std::unique_lock<std::mutex> lk(mu_);
          cv_.wait(lk, [this] { return stop_ || !tasks_.empty(); });
          if (tasks_.empty()) return;
          task = std::move(tasks_.front());
          tasks_.pop_front();
        }
        task();
      }
    });
}

ThreadPool::~ThreadPool() {
  {
    std::lock_guard<std::mutex> g(mu_);
    stop_ = true;
  }
  cv_.notify_all();
  for (auto& w : workers_) w.join();
}

void ThreadPool::submit(std::function<void()> task) {
  {
    std::lock_guard<std::mutex> g(mu_);
    tasks_.push_back(std::move(task));
  }
  cv_.notify_one();
}

void Latch::add(int64_t n) {
  std::lock_guard<std::mutex> g(mu_);
  n_ += n;
}

void Latch::done() {
  std::lock_guard<std::mutex> g(mu_);
  if (--n_ == 0) cv_.notify_all();
}

void Latch::wait() {
  std::unique_lock<std::mutex> lk(mu_);
  cv_.wait(lk, [this] { return n_ == 0; });
}

void host_rerank_rows(const float* X, int64_t n, int d, const float* q, const uint64_t* cand, int R,
                      const int32_t* rowk, int k_stride, int64_t q0, int64_t q1, int64_t* ids,
                      float* dist) {
  std::vector<std::pair<double, int64_t>> c;
  c.reserve(R);
  // the rows are random in host memory: request the rows of the candidates
  // kAhead positions ahead while the current one is summed
  constexpr int kAhead = 12;
  const size_t row_bytes = (size_t)d * sizeof(float);
  auto prefetch_row = [&](uint64_t key) {
    if (key == KEY_NONE || (int64_t)(uint32_t)key >= n) return;
    const char* x = reinterpret_cast<const char*>(X + (int64_t)(uint32_t)key * d);
    for (size_t b = 0; b < row_bytes; b += 64) __builtin_prefetch(x + b, 0, 0);
  };
  for (int64_t i = q0; i < q1; ++i) {
    const float* qi = q + i * d;
    c.clear();
    for (int r = 0; r < std::min(R, kAhead); ++r) prefetch_row(cand[i * R + r]);
    for (int r = 0; r < R; ++r) {
      if (r + kAhead < R) prefetch_row(cand[i * R + r + kAhead]);
      const uint64_t key = cand[i * R + r];
      if (key == KEY_NONE) continue;
      const int64_t id = (int64_t)(uint32_t)key;
      if (id >= n) continue;  // never read outside X
      const float* x = X + id * d;
      // eight independent FP64 partial sums (dimension t goes to sum t % 8),
      // added pairwise at the end: the order is fixed, and without one serial
      // chain of dependent additions a row costs a few vector operations
      double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int t = 0;
      for (; t + 8 <= d; t += 8)
        for (int j = 0; j < 8; ++j) {
          const double diff = (double)qi[t + j] - (double)x[t + j];
          acc[j] += diff * diff;
        }
      for (int j = 0; t < d; ++t, ++j) {
        const double diff = (double)qi[t] - (double)x[t];
        acc[j] += diff * diff;
      }
      const double s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
      c.emplace_back(s, id);
    }
    const int k = rowk ? rowk[i] : k_stride;
    const int m = std::min<int>(k, (int)c.size());
    std::partial_sort(c.begin(), c.begin() + m, c.end());
    for (int t = 0; t < k_stride; ++t) {
      ids[i * k_stride + t] = t < m ? c[t].second : -1;
      dist[i * k_stride + t] = t < m ? (float)c[t].first : INFINITY;
    }
  }
}

}  // namespace rbq
