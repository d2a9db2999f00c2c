// Batched search whose device workspace is never allocated: it lives in a
// fixed device array of this library, one copy per GPU, for callers that
// cannot allocate device memory (work recorded under stream capture, serving
// loops that forbid allocation). The kernels and the schedule are those of
// rbq_search; only where the workspace comes from differs.
#include <mutex>

#include "index.hpp"

namespace rbq {

namespace {

constexpr size_t kNoAllocBytes = (size_t)256 << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

// The workspace array. Each GPU that uses it holds its own copy, from the
// first call on that GPU until the process ends. Host code never hands the
// array's name to a kernel or a copy (on the host it is only a stand-in): it
// uses the device address that hipGetSymbolAddress returns for the current
// device, kept per device below.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
char* g_addr[kMaxDevices] = {};

// The array's address on `dev`, looked up once per device with it current.
char* scratch_on(int dev) {
  RBQ_CHECK(dev >= 0 && dev < kMaxDevices, "rbq_search_noalloc: device ordinal out of range");
  std::lock_guard<std::mutex> g(g_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    RBQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) fail(RBQ_EDEVICE, "rbq_search_noalloc: no device address for the workspace array");
    g_addr[dev] = static_cast<char*>(p);
  }
  return g_addr[dev];
}

}  // namespace

size_t noalloc_scratch_bytes() { return kNoAllocBytes; }

void search_noalloc(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids,
                    float* dist, hipStream_t s) {
  RBQ_CHECK(!idx->vectors_on_host,
            "rbq_search_noalloc: the index must keep its raw vectors in HBM (the host re-rank "
            "stages candidates in pinned host memory)");
  if (nq == 0) return;
  RBQ_CHECK(is_device_ptr(q) && is_device_ptr(ids) && is_device_ptr(dist),
            "rbq_search_noalloc: q, ids and sqdist must be device pointers");
  RBQ_HIP(hipSetDevice(idx->device));
  char* base = scratch_on(idx->device);
  // the largest candidate pool whose whole workspace fits the array
  const int64_t budget =
      fit_pool_budget(idx, nq, nprobe, k, R, nq * (int64_t)nprobe, kNoAllocBytes, (int64_t)2 * nq * R * 8);
  if (budget < 0)
    fail(RBQ_EINVAL,
         "rbq_search_noalloc: this batch needs more workspace than the 256 MiB no-allocation array "
         "holds (" + std::to_string(search_workspace_bytes(idx, nq, nprobe, k, R, nq * (int64_t)nprobe,
                                                          (int64_t)2 * nq * R * 8)) +
             " bytes); split it into smaller batches");
  SearchIO io;
  io.pool_budget = budget;
  io.ws_base = base;
  io.ws_cap = kNoAllocBytes;
  io.untimed = true;  // no stage events: nothing is created
  search(idx, q, nq, nprobe, k, R, ids, dist, s, io);
}

}  // namespace rbq
