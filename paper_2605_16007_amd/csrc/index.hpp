// The index object behind the opaque rbq_index handle, and the per-call
// device workspaces.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <atomic>
#include <cstdint>
#include <memory>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "host_rerank.hpp"
#include "kernels.hpp"
#include "rbq.h"

namespace rbq {

// HIP events of one timed search (read back lazily by rbq_get_timings).
struct TimingRec {
  hipEvent_t e[6] = {};           // start, probe, rotate, quant, scan+merge, rerank
  std::vector<hipEvent_t> scan;   // (start, end) around every scan launch
  std::vector<char> scan_lm;      // per launch: 0 query-major popcount, 1 list-major, 2 fused
  int64_t group = 0, popc = 0;    // scan launches: list-major; query-major (popcount or fused)
  int64_t fused = 0;              // of the query-major launches, the fused ones
  bool first_part = true;         // the first (or only) part of one search
};

// Launch choices of a search that leave its results unchanged (the autotuner
// measures them per batch shape). scan: 1 query-major everywhere, 2 the
// list-major MFMA scan for chunks of probe ranks with >= gm * nlist (query,
// probe) pairs (gm = 0: all chunks) and query-major for the others; G: queries
// per list-major item; wg_per_cu: persistent list-major workgroups per CU;
// first_factor: the first chunk holds about first_factor * R candidates per
// query; growth: each later chunk is (growth - 1) times the prefix scanned.
struct TuneCfg {
  int scan = 0, G = 64, wg_per_cu = 8, first_factor = 2, gm = 4, growth = 2;
  int early = 0;  // chunks before the list-major ones: 0 fused scan+select, 1 popcount scan + merge
  int B = 0;      // list-major items over index blocks of B micro-blocks (0: whole lists)
  int merge = 0;  // pool merges on 256-thread workgroups: 0 none, 1 after the first list-major chunk, 2 all
};

// A device scratch area reused across calls. `done` is recorded on the stream
// of the call that last used it; the area is handed out again only once that
// event has completed, so concurrent calls on distinct streams never share one.
struct Workspace {
  char* base = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  ~Workspace();
};

// Carves aligned sub-buffers out of a workspace.
struct Carver {
  char* base;
  size_t off = 0;
  explicit Carver(char* b) : base(b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

// Device memory owned by the index; freed with it.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void alloc(size_t b);
  void reset();
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace rbq

struct rbq_index {
  int device = 0;
  int64_t n = 0;
  int d = 0, ld = 0, nlist = 0, bq = 4, bqs = 4, W = 0;
  int vectors_on_host = 0;
  int host_threads = 0;
  int64_t nmb = 0;            // micro-blocks over all lists
  int64_t max_list_len = 0;

  // device arrays
  rbq::DevBuf X;       // n x ld raw vectors in id order (vectors_on_host == 0, FP32 form)
  rbq::DevBuf X8;      // the same as n x ld bytes when every value is an integer in [0, 255]
  rbq::DevBuf C;       // nlist x ld centroids
  rbq::DevBuf Crot;    // nlist x ld rotated centroids P^T c
  rbq::DevBuf cnorm;   // nlist, ||c||^2
  rbq::DevBuf Pt;      // d x ld, row i = column i of P
  rbq::DevBuf blocks;  // nmb micro-block records
  rbq::DevBuf list_mb, list_len, pos2id;
  rbq::DevBuf nx, alpha;  // per position, for export
  rbq::DevBuf flat;       // IVF-Flat records: per micro-block dp rows of 64 floats + 64 ||x||^2

  // host copies
  std::vector<float> hC;          // nlist x d
  std::vector<float> hP;          // d x d row-major
  std::vector<int32_t> h_assign;  // n
  std::vector<int32_t> h_list_len, h_list_mb, h_pos2id;
  float* hostX = nullptr;         // n x d host rows when vectors_on_host
  size_t hostX_mapped = 0;        // bytes mapped for the index's own rows
  bool hostX_owned = true;        // false: the caller's rows (borrow_vectors)

  // options (rbq_set_option) and device facts
  std::atomic<int> opt_scan{0};
  std::atomic<int> opt_group_min{4};
  std::atomic<int64_t> opt_pool_cap{0};
  std::atomic<int> opt_rotation{0};  // 0 FP32, 1 BF16 inputs (FP32 accumulation)
  std::atomic<int> opt_group_size{0};  // queries per list-major item (0: tuned or built-in)
  std::atomic<int> opt_estimator{0};   // 0 B_q-bit query, 1 unquantised FP32 residual, 2 IVF-Flat
  std::atomic<int> opt_block{-1};      // micro-blocks per list-major index block (-1: tuned or built-in)
  std::atomic<int> opt_host_parts{0};  // sub-batches of a host re-rank search (0: automatic)
  // autotuned launch choices per batch-shape bucket (rbq_autotune)
  std::mutex tune_mu;
  std::map<uint64_t, rbq::TuneCfg> tune;
  int num_cus = 256;
  int64_t device_mem = 0;  // bytes of device memory (sizes the default pool budget)

  // per-call scratch
  std::mutex ws_mu;
  std::vector<std::unique_ptr<rbq::Workspace>> ws_free;

  // stage timing: sums over the timed searches since timing was enabled.
  // Each timed search leaves its stage events in `pending`; they are read
  // (and destroyed) by rbq_get_timings, so no search waits for them.
  std::atomic<int> timing{0};
  std::mutex timing_mu;
  rbq_timings last{};
  std::vector<rbq::TimingRec> pending;
  rbq::DevBuf tcounter;  // device sums: scanned vectors, record bytes read; the same two
                         // for the list-major launches alone, then for the fused ones;
                         // then the queries redone after a pool overflow

  // host re-rank (vectors_on_host): worker threads and pinned staging, made on
  // first use and kept with the index
  std::mutex host_mu;
  std::unique_ptr<rbq::ThreadPool> pool;
  // the GPU parts of host re-rank searches run on one stream of the index,
  // each search's parts queued whole (host_gpu_mu): concurrent callers then
  // take turns on the GPU and one's host re-rank overlaps the next one's
  // GPU work instead of both halves running side by side at half speed
  hipStream_t host_gpu_stream = nullptr;
  // the candidate hand-off of those parts (device to pinned host memory) runs
  // on a stream of its own, so the next part's kernels do not queue behind it
  hipStream_t host_copy_stream = nullptr;
  std::mutex host_gpu_mu;
  std::vector<std::pair<void*, size_t>> pinned_free;

  ~rbq_index();
};

namespace rbq {

std::unique_ptr<Workspace> ws_acquire(rbq_index* idx, size_t bytes);
void ws_release(rbq_index* idx, std::unique_ptr<Workspace> ws, hipStream_t s);

bool is_device_ptr(const void* p);
// Host rows of the CPU re-rank: 2 MiB-aligned anonymous memory advised for
// transparent huge pages (not pinned); filled by several threads.
float* host_rows_alloc(size_t bytes, size_t* mapped);
void host_rows_free(float* p, size_t mapped);
void host_rows_fill(float* dst, const float* src, size_t count, int threads);
void upload_rows(float* dst, int ld, const float* src, int d, int64_t n, hipStream_t s);

rbq_index* build_index(const float* x, int64_t n, int d, const rbq_build_params& p);
// Keeps idx->X as bytes (idx->X8) when every raw value is an integer in [0, 255].
void compact_raw_vectors(rbq_index* idx, hipStream_t s);

struct SearchIO {
  const rbq_debug_io* dbg = nullptr;  // stage injection / outputs (host pointers)
  // mixed batches (host arrays of nq): query i probes q_nprobe[i] <= nprobe
  // lists, keeps q_R[i] <= R candidates and returns q_k[i] <= k results (its
  // output row, of stride k, is padded with (-1, +inf))
  const int32_t* q_nprobe = nullptr;
  const int32_t* q_k = nullptr;
  const int32_t* q_R = nullptr;
  int64_t pool_budget = 0;  // bytes for the candidate rows (0: 512 MB)
  const TuneCfg* force = nullptr;  // launch choices to use (autotuner trials)
  bool continues_search = false;   // a later sub-batch of a search already counted
  // caller-owned device scratch (else the index's pool); not reused by the
  // caller before the search's stream has passed this call
  char* ws_base = nullptr;
  size_t ws_cap = 0;
  bool untimed = false;  // never record stage events (no event creation)
};
// Workspace bytes of a mixed search of nq queries (nprobe, k, R the batch's
// largest, scanned_pairs the sum of per-query nprobe) with that pool budget.
size_t search_workspace_bytes(const rbq_index* idx, int64_t nq, int nprobe, int k, int R,
                              int64_t scanned_pairs, int64_t pool_budget);
// The largest pool budget >= lo whose workspace (search_workspace_bytes) fits
// in cap bytes; -1 if not even lo fits.
int64_t fit_pool_budget(const rbq_index* idx, int64_t nq, int nprobe, int k, int R,
                        int64_t scanned_pairs, size_t cap, int64_t lo);
void search(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids,
            float* dist, hipStream_t s, const SearchIO& io);
// Sub-batches a search with the re-rank on host cores is cut into: while the
// host re-ranks one, the GPU searches the next.
int host_rerank_parts(const rbq_index* idx, int64_t nq, int nprobe);
// Phases 1-4 only: the coarse top-R of every query (nq x R sort keys) is
// copied into cand_host, and the queries into q_host when q is on the device
// (both pinned host memory); returns when they are there. The re-rank's input.
void search_candidates(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R,
                       uint64_t* cand_host, float* q_host, hipStream_t s, const SearchIO& io);
// rbq_search on the library's fixed per-GPU workspace array (noalloc.hip).
void search_noalloc(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids,
                    float* dist, hipStream_t s);
size_t noalloc_scratch_bytes();

// Autotuner (tune.cpp): bucket key of a batch shape, the table lookup used by
// every search, trials, and the text cache.
uint64_t tune_key(int64_t nq, int nprobe, int R);
bool tune_lookup(rbq_index* idx, int64_t nq, int nprobe, int R, TuneCfg* out);
void autotune(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R,
              rbq_tune_result* out);
void tune_save(rbq_index* idx, const char* path);
int tune_load(rbq_index* idx, const char* path);

void export_item(const rbq_index* idx, int what, void* dst, size_t bytes);
void save_index(const rbq_index* idx, const char* path);
rbq_index* load_index(const char* path);

}  // namespace rbq
