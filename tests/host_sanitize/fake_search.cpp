// Host-only stand-ins for the device side of the library, for the thread
// sanitizer build of the serving loop: a "search" that writes a result every
// query can be checked by (ids derived from the query and the rank), and the
// workspace sizing the lanes use for admission.
#include <algorithm>

#include "index.hpp"

namespace rbq {

Workspace::~Workspace() {}
void DevBuf::alloc(size_t b) { reset(); p = std::malloc(b ? b : 1); bytes = b; }
void DevBuf::reset() { std::free(p); p = nullptr; bytes = 0; }
bool is_device_ptr(const void*) { return false; }

size_t search_workspace_bytes(const rbq_index*, int64_t nq, int nprobe, int k, int R, int64_t pairs,
                              int64_t pool_budget) {
  return (size_t)(nq * (int64_t)(k + R) * 12 + pairs * 2048 + std::max<int64_t>(0, pool_budget) / 4 + 4096);
}

int64_t fit_pool_budget(const rbq_index* idx, int64_t nq, int nprobe, int k, int R, int64_t pairs,
                        size_t cap, int64_t lo) {
  if (search_workspace_bytes(idx, nq, nprobe, k, R, pairs, lo) > cap) return -1;
  int64_t b = lo;
  while (search_workspace_bytes(idx, nq, nprobe, k, R, pairs, 2 * b) <= cap && b < ((int64_t)1 << 40)) b *= 2;
  return b;
}

// Result of query i: ids q[0] * 1000 + r and distances r for its own k, the
// rest of the row (-1, +inf), after touching the caller's workspace.
void search(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids, float* dist,
            hipStream_t, const SearchIO& io) {
  RBQ_CHECK(io.ws_base && search_workspace_bytes(idx, nq, nprobe, k, R, nq * (int64_t)nprobe, io.pool_budget) <=
                              io.ws_cap + (size_t)io.pool_budget,
            "fake search: workspace too small");
  std::memset(io.ws_base, 0, std::min<size_t>(io.ws_cap, 4096));
  for (int64_t i = 0; i < nq; ++i) {
    const int ki = io.q_k ? io.q_k[i] : k;
    for (int r = 0; r < k; ++r) {
      ids[i * k + r] = r < ki ? (int64_t)q[i * idx->d] * 1000 + r : -1;
      dist[i * k + r] = r < ki ? (float)r : INFINITY;
    }
  }
}

}  // namespace rbq

rbq_index::~rbq_index() {}
