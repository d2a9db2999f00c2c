// Batched search (Sec. 3.1.2): Phase 1 probe, query rotation and B_q-bit
// quantisation, Phase 3 code scan with the fused estimator, Phase 4 top-R,
// Phase 5 exact re-rank.
#include <algorithm>
#include <array>
#include <vector>
#include <cstring>

#include "index.hpp"
#include "host_rerank.hpp"

namespace rbq {

namespace {

// Timing counters: acc[0] += sum of list sizes over the pairs of probe ranks
// [p0, p0 + pn); acc[1] += their padded record bytes when `qm` (each
// query-major item reads its whole list).
// (instrumented searches) the queries flagged for a redo
__global__ void k_count_flags(const uint32_t* flags, int n, unsigned long long* acc) {
  __shared__ unsigned long long part[256];
  unsigned long long c = 0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < n; t += gridDim.x * 256) c += flags[t] ? 1u : 0u;
  part[threadIdx.x] = c;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, part[0]);
}

__global__ void k_count_scanned(const int32_t* probes, const int32_t* list_len, int nq, int nprobe,
                                int p0, int pn, int rec_bytes, int qm, unsigned long long* acc) {
  __shared__ unsigned long long part[2][256];
  unsigned long long s = 0, b = 0;
  const int64_t pairs = (int64_t)nq * pn;
  for (int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x; t < pairs; t += (int64_t)gridDim.x * 256) {
    const int64_t i = t / pn;
    const int j = probes[i * nprobe + p0 + (t - i * pn)];
    const int len = j >= 0 ? list_len[j] : 0;
    s += (unsigned long long)len;
    if (qm) b += (unsigned long long)((len + 63) / 64) * 64 * rec_bytes;
  }
  part[0][threadIdx.x] = s;
  part[1][threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      part[0][threadIdx.x] += part[0][threadIdx.x + off];
      part[1][threadIdx.x] += part[1][threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(&acc[0], part[0][0]);
    atomicAdd(&acc[1], part[1][0]);
  }
}

// acc += padded record bytes of every list-major item (items x list bytes)
__global__ void k_count_group_bytes(const int32_t* cnt, const int32_t* list_len, int nlist, int G,
                                    int rec_bytes, unsigned long long* acc) {
  __shared__ unsigned long long part[256];
  unsigned long long b = 0;
  for (int j = blockIdx.x * 256 + threadIdx.x; j < nlist; j += gridDim.x * 256)
    b += (unsigned long long)((cnt[j] + G - 1) / G) * ((list_len[j] + 63) / 64) * 64 * rec_bytes;
  part[threadIdx.x] = b;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) part[threadIdx.x] += part[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicAdd(acc, part[0]);
}

struct Bufs {
  float* qpad = nullptr;
  float* score = nullptr;
  int32_t* probes = nullptr;
  float* pscore = nullptr;
  float* qrot = nullptr;
  uint32_t* planes = nullptr;
  uint8_t* qu = nullptr;
  uint8_t* qu8 = nullptr;  // fp8 operand rows of the fp4 x fp8 list-major scan
  float4* scal = nullptr;
  uint8_t* inj_qu = nullptr;
  float* inj_scal = nullptr;
  uint32_t* qthr = nullptr;
  uint32_t* pcnt = nullptr;
  int32_t* gcnt = nullptr;         // list-major map: pairs per (chunk, list) bin
  int32_t* gfill = nullptr;        // list-major map: fill cursor per bin
  int32_t* gbase = nullptr;        // list-major map: first slot per bin
  int32_t* wpart = nullptr;        // list-major map: workgroup sums, then bases
  int32_t* chunk_items = nullptr;  // list-major map: item range of every chunk
  int32_t* slots = nullptr;
  int4* items = nullptr;
  uint32_t* overflow = nullptr;
  uint32_t* counter = nullptr;
  uint64_t* cand = nullptr;
  int32_t* dump_ip = nullptr;
  float* dump_est = nullptr;
  int64_t* ids = nullptr;
  float* dist = nullptr;
  int32_t* spec = nullptr;  // mixed batches: [3][nq] nprobe, k, rerank_n per query
};

struct Chunk {
  int p0, pn;
  bool lm = false;     // list-major MFMA scan (else query-major popcount)
  bool fused = false;  // query-major, scan and selection in one launch
};

// What a search call does and needs, fixed before any launch.
struct Plan {
  int64_t nq = 0, pairs = 0, maxlen = 1;
  int nprobe = 0, k = 0, R = 0;
  int pch = 1, first = 1;
  int64_t cand_ld = 0, pool_cap = 0;
  bool need_qcopy = true, ids_dev = false, dist_dev = false;
  bool inj_probes = false, inj_qu = false, dumps = false, mixed = false, any_group = false;
  bool unq = false;   // unquantised residual (table-lookup query-major scan)
  bool flat = false;  // IVF-Flat: exact distances of the lists' raw rows (list-major)
  GroupChunks gc;  // the list-major chunks (a suffix of the probe ranks)
  int G = 64, wg_per_cu = 8;
  int B = 0;       // micro-blocks per index block of a list-major item (0: whole lists)
  int merge = 0;   // which pool merges run on 256-thread workgroups (TuneCfg::merge)
  const rbq_debug_io* dbg = nullptr;
  std::vector<Chunk> chunks, qm_chunks;
};

// Candidate pools of a search without a memory budget: 1/64 of the device's
// memory, from 512 MiB to 8 GiB (4.5 GB on a 288 GB MI355X). A pool that
// overflows sends its query to an exact redo from scratch, so room is cheaper
// than a redo.
int64_t default_pool_budget(const rbq_index* idx) {
  return std::min<int64_t>((int64_t)8 << 30, std::max<int64_t>((int64_t)512 << 20, idx->device_mem / 64));
}
// batches at least this large scan their query-major chunks with the fused
// one-workgroup-per-query kernel (enough workgroups to fill the GPU)
constexpr int64_t kFusedMinQueries = 128;

// Probe ranks are scanned in chunks: scan items append survivors to their
// query's pool (row layout: R running keys, then the pool), and a merge after
// each chunk folds the pool into the running top-R and lowers the query's
// threshold to its exact R-th estimate, so later chunks keep only candidates
// that can still enter the top-R (the IVF-aware pruning of Sec. 3.3.3).
//
// With d <= 256 each chunk is (growth - 1) times the prefix already scanned
// (growth 2: doubling; the first holds about first_factor * R candidates per
// query), so with the threshold at the exact R-th estimate of that prefix a
// pool expects about (growth - 1) R survivors per chunk. Each chunk picks its scan: the list-major MFMA scan once each probed
// list is shared by >= gm queries of the chunk on average (it reads a list
// once per group of queries), the query-major popcount scan before (each of
// its items keeps at most R survivors, so those chunks are cut to fit the
// pool). A query whose pool overflows in a list-major chunk is searched again,
// from scratch, by the query-major scan (exact; checked once per search).
// Otherwise (query-major only) chunks double from `first` (enough items to
// fill the GPU) up to `pch`, the most probe ranks whose worst case (R keys per
// item) fits the pool budget.
Plan make_plan(const rbq_index* idx, int64_t nq, int nprobe, int k, int R, int64_t scanned_pairs,
               int64_t pool_budget, const rbq_debug_io* dbg, const TuneCfg* force) {
  Plan P;
  P.nq = nq;
  P.nprobe = nprobe;
  P.k = k;
  P.R = R;
  P.pairs = nq * nprobe;
  P.dbg = dbg;
  P.maxlen = std::max<int64_t>(1, idx->max_list_len);
  P.inj_probes = dbg && dbg->inject_probes;
  P.inj_qu = dbg && dbg->inject_qu && idx->opt_estimator.load() != 1;
  P.dumps = dbg && (dbg->ip || dbg->est);
  P.unq = idx->opt_estimator.load() == 1;
  P.flat = idx->opt_estimator.load() == 2 && idx->flat.p != nullptr;
  const int64_t budget = pool_budget > 0 ? pool_budget : default_pool_budget(idx);
  P.pch = (int)std::max<int64_t>(
      1, std::min<int64_t>(nprobe, budget / std::max<int64_t>(1, nq * R * 8) - 1));
  P.first = (int)std::min<int64_t>(P.pch, std::max<int64_t>(1, (2048 + nq - 1) / nq));
  if (dbg && dbg->probe_chunk > 0) P.pch = P.first = std::min(P.pch, (int)dbg->probe_chunk);

  // launch choices: forced (autotuner trial), else tuned for this batch shape,
  // else the built-in rule; an explicit RBQ_OPT_SCAN wins over a tuned form
  TuneCfg cfg;
  bool tuned = false;
  if (force) {
    cfg = *force;
    tuned = true;
  } else {
    tuned = tune_lookup(const_cast<rbq_index*>(idx), nq, nprobe, R, &cfg);
  }
  P.G = idx->opt_group_size.load() > 0 ? idx->opt_group_size.load() : cfg.G;
  if (P.flat) P.G = std::min(P.G, 32);  // two 16-query tiles per IVF-Flat item
  P.B = idx->opt_block.load() >= 0 ? idx->opt_block.load() : cfg.B;
  P.merge = cfg.merge;
  P.wg_per_cu = cfg.wg_per_cu;
  // scan form per chunk of probe ranks: query-major (1) everywhere, or the
  // list-major MFMA scan for every chunk whose (query, probe) pairs number at
  // least gm * nlist (a list is probed by >= gm queries of the chunk on
  // average; gm = 0: every chunk)
  const int opt = idx->opt_scan.load();
  int scan_mode = opt, gm = idx->opt_group_min.load();
  if (force || (opt == 0 && tuned)) {
    scan_mode = cfg.scan;
    gm = cfg.gm;
  } else if (opt == 2) {
    gm = 0;
  } else if (opt == 0) {
    scan_mode = 2;
  }
  // a pool holds a query-major chunk's R keys per probe, and at least the
  // longest list (a first list-major chunk, taken before any threshold, then
  // fits) when the budget allows
  P.pool_cap = (int64_t)R * P.pch;
  if (P.maxlen > P.pool_cap && nq * (R + P.maxlen) * 8 <= budget) P.pool_cap = P.maxlen;
  // the rest of the budget goes to the pools too: a list-major chunk's
  // survivors may exceed R per probe rank (queries whose first lists leave a
  // loose threshold), and an overflowing query is searched again from
  // scratch by one workgroup
  P.pool_cap = std::max<int64_t>(P.pool_cap, std::min<int64_t>(budget / (8 * std::max<int64_t>(1, nq)) - R,
                                                               (int64_t)1 << 28));
  if (P.flat)  // (no redo for IVF-Flat: as large a pool as the budget holds)
    P.pool_cap = std::max<int64_t>(P.pool_cap, std::max<int64_t>(P.maxlen, budget / (8 * std::max<int64_t>(1, nq)) - R));
  P.cand_ld = R + P.pool_cap;
  if (idx->opt_pool_cap.load() > 0) P.pool_cap = std::min<int64_t>(P.pool_cap, idx->opt_pool_cap.load());
  for (int p0 = 0, pn = P.first; p0 < nprobe; p0 += pn, pn = std::min(2 * pn, P.pch)) {
    pn = std::min(pn, nprobe - p0);
    P.qm_chunks.push_back({p0, pn, false, false});
  }
  // (list-major survivors carry their position in the list in 26 bits)
  if (P.unq) scan_mode = 1;  // the unquantised estimator has the query-major scan only
  if (P.flat) {              // IVF-Flat: the list-major scan for every chunk
    scan_mode = 2;
    gm = 0;
  }
  const bool lm_ok = scan_mode == 2 && group_k_steps(idx->d) <= 4 &&
                     idx->max_list_len < (int64_t(1) << 26);
  if (lm_ok) {
    // chunks double the scanned prefix; the first holds about first_factor * R
    // candidates per query on average, and never more than the pool holds
    // even for the longest lists
    const int64_t maxl = std::max<int64_t>(1, idx->max_list_len);
    const int64_t avgl = std::max<int64_t>(1, idx->n / idx->nlist);
    int pn = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nprobe, P.pool_cap / maxl,
                                                          ceil_div((int64_t)cfg.first_factor * R, avgl)}));
    if (dbg && dbg->probe_chunk > 0) pn = std::min(pn, (int)dbg->probe_chunk);
    for (int p0 = 0; p0 < nprobe; p0 += pn, pn = std::max(pn, (cfg.growth - 1) * p0)) {
      pn = std::min(pn, nprobe - p0);
      const int64_t chunk_pairs = scanned_pairs * pn / std::max(1, nprobe);
      // (once list-major, always: the chunk cut at nprobe may be the smaller)
      const bool lm = chunk_pairs >= (int64_t)gm * idx->nlist || (!P.chunks.empty() && P.chunks.back().lm);
      if (lm) {
        P.chunks.push_back({p0, pn, true, false});
        P.any_group = true;
      } else if (nq >= kFusedMinQueries && idx->W <= 32 && cfg.early == 0 && !P.dumps) {
        // (per-vector dumps come from the popcount and list-major scans)
        // one workgroup per query scans and selects in one launch; it lowers
        // its threshold whenever its buffer fills, so consecutive chunks of
        // this kind become one launch
        if (!P.chunks.empty() && P.chunks.back().fused)
          P.chunks.back().pn += pn;
        else
          P.chunks.push_back({p0, pn, false, true});
      } else {  // a query-major chunk appends up to R keys per item: split to fit the pool
        for (int q0 = p0; q0 < p0 + pn; q0 += P.pch)
          P.chunks.push_back({q0, std::min(P.pch, p0 + pn - q0), false, false});
      }
    }
  } else if (scan_mode == 3 && nq >= kFusedMinQueries && idx->W <= 32 && !P.dumps) {
    // one workgroup per query scans and selects over every probe rank in one
    // launch (one work item per query)
    P.chunks.push_back({0, nprobe, false, true});
  } else {
    P.chunks = P.qm_chunks;
  }
  if (P.any_group) {
    // list-major chunks grow with the scanned prefix, so they form a suffix of
    // the ranks; past kMaxGroupChunks of them the last one takes the rest
    size_t f = 0;
    while (!P.chunks[f].lm) ++f;
    if (P.chunks.size() - f > (size_t)kMaxGroupChunks) {
      Chunk& last = P.chunks[f + kMaxGroupChunks - 1];
      last.pn = nprobe - last.p0;
      P.chunks.resize(f + kMaxGroupChunks);
    }
    P.gc.nb = 0;
    for (size_t c = f; c < P.chunks.size(); ++c) {
      RBQ_CHECK(P.chunks[c].lm, "list-major chunks must be a suffix of the probe ranks");
      P.gc.bound[P.gc.nb++] = P.chunks[c].p0;
    }
    P.gc.bound[P.gc.nb] = nprobe;
  }
  return P;
}

void layout(const rbq_index* idx, const Plan& P, Carver& c, Bufs& b) {
  const int64_t nq = P.nq, pairs = P.pairs;
  const int ld = idx->ld, nlist = idx->nlist, W = idx->W, d = idx->d;
  const rbq_debug_io* dbg = P.dbg;
  if (P.need_qcopy) b.qpad = c.take<float>((size_t)nq * ld);
  if (!P.inj_probes) {
    b.score = c.take<float>((size_t)nq * nlist);
  }
  b.probes = c.take<int32_t>(pairs);
  if (dbg && dbg->probe_score) b.pscore = c.take<float>(pairs);
  b.qrot = c.take<float>((size_t)nq * ld);
  const bool codes = !P.unq && !P.flat;  // the quantised query's buffers
  if (codes) b.planes = c.take<uint32_t>((size_t)pairs * W * idx->bqs);
  const bool f8 = codes && P.any_group && group_uses_f8(idx->bq, d);
  if (codes && ((dbg && dbg->qu) || (P.any_group && !f8))) b.qu = c.take<uint8_t>((size_t)pairs * W * 32);
  if (f8) b.qu8 = c.take<uint8_t>((size_t)pairs * 128 * group_f8_steps(d));
  if (P.any_group) {
    const int64_t bins = (int64_t)P.gc.nb * nlist;
    // cleared together at the start of a search: the overflow flag, the
    // chunks' item cursors, the bins' pair counts and fill cursors
    b.counter = c.take<uint32_t>(1 + kMaxGroupChunks + 2 * bins);
    b.gcnt = reinterpret_cast<int32_t*>(b.counter + 1 + kMaxGroupChunks);
    b.gfill = b.gcnt + bins;
    b.gbase = c.take<int32_t>(bins);
    b.wpart = c.take<int32_t>((size_t)2 * P.gc.nb * group_map_workgroups(nlist));
    b.chunk_items = c.take<int32_t>(kMaxGroupChunks + 1);
    b.slots = c.take<int32_t>(pairs);
    b.items = c.take<int4>(group_map_item_bound(pairs, P.G, P.gc.nb, nlist, idx->nmb, idx->max_list_len, P.B));
    b.overflow = c.take<uint32_t>(nq);
  }
  b.scal = c.take<float4>(pairs);
  if (P.inj_qu) {
    b.inj_qu = c.take<uint8_t>((size_t)pairs * d);
    b.inj_scal = c.take<float>((size_t)pairs * 3);
  }
  b.qthr = c.take<uint32_t>(nq);
  b.pcnt = c.take<uint32_t>(nq);
  b.cand = c.take<uint64_t>((size_t)nq * P.cand_ld);
  if (P.dumps) {
    b.dump_ip = c.take<int32_t>((size_t)pairs * P.maxlen);
    b.dump_est = c.take<float>((size_t)pairs * P.maxlen);
  }
  if (!P.ids_dev) b.ids = c.take<int64_t>((size_t)nq * P.k);
  if (!P.dist_dev) b.dist = c.take<float>((size_t)nq * P.k);
  if (P.mixed) b.spec = c.take<int32_t>((size_t)nq * 3);
}

}  // namespace

}  // namespace rbq

namespace rbq {

size_t search_workspace_bytes(const rbq_index* idx, int64_t nq, int nprobe, int k, int R,
                              int64_t scanned_pairs, int64_t pool_budget) {
  Plan P = make_plan(idx, nq, nprobe, k, R, scanned_pairs, pool_budget, nullptr, nullptr);
  P.mixed = true;
  Carver dry(nullptr);
  Bufs b;
  layout(idx, P, dry, b);
  return dry.off + 256;
}

int64_t fit_pool_budget(const rbq_index* idx, int64_t nq, int nprobe, int k, int R,
                        int64_t scanned_pairs, size_t cap, int64_t lo) {
  lo = std::max<int64_t>(1, lo);
  auto fits = [&](int64_t b) {
    return search_workspace_bytes(idx, nq, nprobe, k, R, scanned_pairs, b) <= cap;
  };
  if (!fits(lo)) return -1;
  // the workspace grows with the pool budget (larger pools, and the chunk
  // schedule that goes with them), so the largest fitting budget is found by
  // bisection; the result is checked, since the schedule's buffers only
  // mostly grow with it
  int64_t good = lo, hi = (int64_t)cap;
  while (good < hi) {
    const int64_t mid = good + (hi - good + 1) / 2;
    if (fits(mid))
      good = mid;
    else
      hi = mid - 1;
  }
  return fits(good) ? good : lo;
}

namespace {

// Host re-rank hand-off of one (sub-)batch: the candidate rows and the
// queries staged in pinned host memory, ready once `ready` has passed.
struct HostJob {
  uint64_t* cand = nullptr;  // nq x R keys (written by the search)
  float* qh = nullptr;       // nq x d queries (written by the search when it has them on the device)
  hipEvent_t ready = nullptr;
  // (optional) the stream that copies them out, and an event that orders it
  // after the search's kernels; the search's workspace is then released on it
  hipStream_t copy = nullptr;
  hipEvent_t staged = nullptr;
};

// Pinned host memory from the index's free list (returned on destruction).
struct Pinned {
  rbq_index* idx;
  void* p = nullptr;
  size_t cap = 0;
  Pinned(rbq_index* ix, size_t bytes) : idx(ix) {
    {
      std::lock_guard<std::mutex> g(idx->host_mu);
      size_t best = (size_t)-1;
      for (size_t i = 0; i < idx->pinned_free.size(); ++i)
        if (idx->pinned_free[i].second >= bytes &&
            (best == (size_t)-1 || idx->pinned_free[i].second < idx->pinned_free[best].second))
          best = i;
      if (best != (size_t)-1) {
        p = idx->pinned_free[best].first;
        cap = idx->pinned_free[best].second;
        idx->pinned_free.erase(idx->pinned_free.begin() + best);
        return;
      }
    }
    RBQ_HIP(hipHostMalloc(&p, bytes, hipHostMallocDefault));
    cap = bytes;
  }
  ~Pinned() {
    std::lock_guard<std::mutex> g(idx->host_mu);
    idx->pinned_free.emplace_back(p, cap);
  }
};

void search_part(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids,
                 float* dist, hipStream_t s, const SearchIO& io, HostJob* job) {
  if (nq == 0) return;
  RBQ_HIP(hipSetDevice(idx->device));
  const int d = idx->d, ld = idx->ld, nlist = idx->nlist, W = idx->W, bqs = idx->bqs;
  const rbq_debug_io* dbg = io.dbg;
  const bool mixed = io.q_nprobe != nullptr;
  int64_t scanned_pairs = nq * (int64_t)nprobe;
  if (mixed) {
    RBQ_CHECK(io.q_k && io.q_R, "mixed batch needs nprobe, k and rerank_n per query");
    scanned_pairs = 0;
    for (int64_t i = 0; i < nq; ++i) {
      RBQ_CHECK(io.q_nprobe[i] >= 1 && io.q_nprobe[i] <= nprobe, "per-query nprobe out of range");
      RBQ_CHECK(io.q_R[i] >= 1 && io.q_R[i] <= R, "per-query rerank_n out of range");
      RBQ_CHECK(io.q_k[i] >= 1 && io.q_k[i] <= k && io.q_k[i] <= io.q_R[i], "per-query k out of range");
      scanned_pairs += io.q_nprobe[i];
    }
  }
  Plan P = make_plan(idx, nq, nprobe, k, R, scanned_pairs, io.pool_budget, dbg, io.force);
  P.mixed = mixed;
  const bool qdev = is_device_ptr(q);
  P.need_qcopy = !qdev || ld != d || (reinterpret_cast<uintptr_t>(q) & 15);
  P.ids_dev = ids && is_device_ptr(ids);
  P.dist_dev = dist && is_device_ptr(dist);
  const bool need_qcopy = P.need_qcopy, ids_dev = P.ids_dev, dist_dev = P.dist_dev;
  const int64_t pairs = P.pairs;
  const bool inj_probes = P.inj_probes, inj_qu = P.inj_qu, dumps = P.dumps;
  const int64_t maxlen = P.maxlen;
  const bool timed = !io.untimed && idx->timing.load() != 0;
  // bytes of one vector's record: code words and two factors, or for
  // IVF-Flat its full-precision row and squared norm
  const int rec_bytes = P.flat ? (flat_dp(d) + 1) * 4 : W * 4 + 8;
  const int64_t cand_ld = P.cand_ld;
  const int64_t pool_cap = P.pool_cap;
  const bool any_group = P.any_group;
  const std::vector<Chunk>& chunks = P.chunks;
  const std::vector<Chunk>& qm_chunks = P.qm_chunks;
  Bufs b;
  {
    Carver dry(nullptr);
    layout(idx, P, dry, b);
    b = Bufs();
    std::unique_ptr<Workspace> ws;
    char* base = io.ws_base;
    if (base) {
      RBQ_CHECK(dry.off + 256 <= io.ws_cap, "caller workspace too small for this batch");
      base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(base) + 255) & ~uintptr_t(255));
    } else {
      ws = ws_acquire(idx, dry.off + 256);
      base = ws->base;
    }
    Carver c(base);
    layout(idx, P, c, b);
    const int32_t* d_np = nullptr;
    const int32_t* d_k = nullptr;
    const int32_t* d_R = nullptr;
    if (mixed) {
      RBQ_HIP(hipMemcpyAsync(b.spec, io.q_nprobe, nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
      RBQ_HIP(hipMemcpyAsync(b.spec + nq, io.q_k, nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
      RBQ_HIP(hipMemcpyAsync(b.spec + 2 * nq, io.q_R, nq * sizeof(int32_t), hipMemcpyHostToDevice, s));
      d_np = b.spec;
      d_k = b.spec + nq;
      d_R = b.spec + 2 * nq;
    }

    // stage events: start, probe, rotate, quant, scan+merge loop, rerank; plus
    // a (start, end) pair around every scan launch
    TimingRec tr;
    auto newev = [&]() {
      hipEvent_t e;
      RBQ_HIP(hipEventCreate(&e));
      return e;
    };
    if (timed)
      for (auto& e : tr.e) e = newev();
    auto mark = [&](int i) {
      if (timed) RBQ_HIP(hipEventRecord(tr.e[i], s));
    };

    const float* qd = q;
    if (need_qcopy) {
      // (a fill kernel: no memset node when the caller captures the stream)
      if (ld != d) launch_fill_u32(s, reinterpret_cast<uint32_t*>(b.qpad), 0u, nq * ld);
      upload_rows(b.qpad, ld, q, d, nq, s);
      qd = b.qpad;
    }
    mark(0);
    // Phase 1: probe scores ||c||^2 - 2<q,c> on MFMA, then top-nprobe per query
    if (inj_probes) {
      for (int64_t t = 0; t < pairs; ++t)
        RBQ_CHECK(dbg->inject_probes[t] >= 0 && dbg->inject_probes[t] < nlist, "injected probe out of range");
      RBQ_HIP(hipMemcpyAsync(b.probes, dbg->inject_probes, pairs * sizeof(int32_t), hipMemcpyHostToDevice, s));
    } else {
      launch_gemm_tn(s, 1, qd, ld, idx->C.as<float>(), ld, b.score, nlist, (int)nq, nlist, ld,
                     idx->cnorm.as<float>());
      TopkArgs ta;
      ta.score = b.score;
      ta.ld = nlist;
      ta.ncols = nlist;
      ta.k = nprobe;
      ta.out_low = b.probes;
      ta.out_val = b.pscore;
      launch_row_topk(s, ta, (int)nq);
    }
    if (mixed) launch_mask_probes(s, b.probes, (int)nq, nprobe, d_np);
    mark(1);
    // query rotation q' = P^T q (row form q P) on MFMA
    if (idx->opt_rotation.load() == 1)
      launch_gemm_tn_bf16(s, qd, ld, idx->Pt.as<float>(), ld, b.qrot, ld, (int)nq, d, ld);
    else
      launch_gemm_tn(s, 0, qd, ld, idx->Pt.as<float>(), ld, b.qrot, ld, (int)nq, d, ld, nullptr);
    if (dbg && dbg->inject_qrot)  // (rows of d floats into rows of ld; the padding stays zero)
      RBQ_HIP(hipMemcpy2DAsync(b.qrot, ld * sizeof(float), dbg->inject_qrot, d * sizeof(float),
                               d * sizeof(float), nq, hipMemcpyHostToDevice, s));
    mark(2);
    // residual quantisation per (query, probe)
    if (inj_qu) {
      RBQ_HIP(hipMemcpyAsync(b.inj_qu, dbg->inject_qu, (size_t)pairs * d, hipMemcpyHostToDevice, s));
      RBQ_CHECK(dbg->inject_scalars != nullptr, "inject_qu needs inject_scalars");
      RBQ_HIP(hipMemcpyAsync(b.inj_scal, dbg->inject_scalars, (size_t)pairs * 3 * sizeof(float),
                             hipMemcpyHostToDevice, s));
    }
    if (dumps) {
      RBQ_HIP(hipMemsetAsync(b.dump_ip, 0, (size_t)pairs * maxlen * sizeof(int32_t), s));
      RBQ_HIP(hipMemsetAsync(b.dump_est, 0, (size_t)pairs * maxlen * sizeof(float), s));
    }
    if (!P.unq && !P.flat)  // (the unquantised and IVF-Flat scans need no quantised query)
      launch_quant(s, b.qrot, ld, idx->Crot.as<float>(), ld, b.probes, (int)nq, nprobe, d, W, idx->bq,
                   bqs, b.planes, b.qu, b.qu8, 128 * group_f8_steps(d), b.scal, b.inj_qu, b.inj_scal);
    mark(3);
    // Phase 3 + Phase 4: code scan with the estimator and per-item top-R,
    // then the per-query merge, one chunk of probe ranks at a time
    ScanArgs sa;
    sa.L = ListsView{idx->blocks.as<uint32_t>(), idx->list_mb.as<int32_t>(), idx->list_len.as<int32_t>(),
                     idx->pos2id.as<int32_t>(), W, d};
    sa.Q = PairsView{b.planes, b.scal, bqs};
    sa.probes = b.probes;
    sa.nq = (int)nq;
    sa.nprobe = nprobe;
    sa.R = R;
    sa.out_ld = cand_ld;
    sa.qthr = b.qthr;
    sa.out = b.cand;
    sa.dump_ip = b.dump_ip;
    sa.dump_est = b.dump_est;
    sa.maxlen = maxlen;
    sa.qrot = b.qrot;
    sa.ldq = ld;
    sa.crot = idx->Crot.as<float>();
    sa.ldc = ld;
    {
      // running top-R rows empty, thresholds open, pools empty; the list-major
      // bins and cursors cleared
      SearchInit si;
      si.cand = b.cand;
      si.cand_ld = cand_ld;
      si.nq = (int)nq;
      si.R = R;
      si.qthr = b.qthr;
      si.pcnt = b.pcnt;
      if (any_group) {
        si.overflow = b.overflow;
        si.z0 = b.counter;
        si.n0 = 1 + kMaxGroupChunks + 2 * (int64_t)P.gc.nb * nlist;
      }
      launch_search_init(s, si);
    }
    // the (chunk, list) -> pairs map of every list-major chunk
    if (any_group)
      launch_group_map(s, b.probes, (int)nq, nprobe, P.gc, nlist, P.G, P.B, idx->list_mb.as<int32_t>(),
                       idx->list_len.as<int32_t>(),
                       GroupMap{b.gcnt, b.gfill, b.gbase, b.wpart, b.chunk_items, b.slots, b.items});
    sa.pcnt = b.pcnt;
    sa.qmask = nullptr;
    GroupArgs ga;
    ga.L = sa.L;
    ga.qu = b.qu8 ? b.qu8 : b.qu;
    ga.qu_ld = b.qu8 ? 128 * group_f8_steps(d) : W * 32;
    ga.scal = b.scal;
    ga.nq = (int)nq;
    ga.nprobe = nprobe;
    ga.R = R;
    ga.nlist = nlist;
    ga.G = P.G;
    ga.bq = idx->bq;
    ga.slots = b.slots;
    ga.item_off = b.chunk_items;
    ga.items = b.items;
    ga.any_overflow = b.counter;
    ga.qthr = b.qthr;
    ga.pool = b.cand;
    ga.pool_ld = cand_ld;
    ga.cap = (int)pool_cap;
    ga.pcnt = b.pcnt;
    ga.overflow = b.overflow;
    ga.probes = b.probes;
    ga.dump_ip = b.dump_ip;
    ga.dump_est = b.dump_est;
    ga.maxlen = maxlen;
    TopkArgs ma;
    ma.keys = b.cand;
    ma.ld = cand_ld;
    ma.k = R;
    ma.out_keys = b.cand;
    ma.ldo = cand_ld;
    ma.rowcnt = b.pcnt;
    ma.qthr = b.qthr;
    ma.rowk = d_R;
    ma.sorted = false;
    auto scan_popc_chunk = [&](const Chunk& ch) {
      sa.p0 = ch.p0;
      sa.pn = ch.pn;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        e0 = newev();
        e1 = newev();
        tr.scan.push_back(e0);
        tr.scan.push_back(e1);
        RBQ_HIP(hipEventRecord(e0, s));
      }
      if (P.unq)
        launch_scan_lut(s, sa);
      else
        launch_scan_popc(s, sa);
      if (timed) {
        RBQ_HIP(hipEventRecord(e1, s));
        tr.scan_lm.push_back(0);
        tr.popc += 1;
        if (!sa.qmask) {  // (the redo of overflowed queries is not counted)
          hipLaunchKernelGGL(k_count_scanned, dim3(64), dim3(256), 0, s, b.probes,
                             idx->list_len.as<int32_t>(), (int)nq, nprobe, ch.p0, ch.pn, rec_bytes, 1,
                             idx->tcounter.as<unsigned long long>());
          RBQ_HIP(hipGetLastError());
        }
      }
      ma.max_extra = R * ch.pn;
      ma.merge_threads = P.merge == 2 ? 256 : 512;
      launch_row_topk(s, ma, (int)nq);
    };
    int lm_chunk = 0;  // index of the next list-major chunk
    auto scan_group_chunk = [&](const Chunk& ch) {
      const int c = lm_chunk++;
      RBQ_CHECK(c < P.gc.nb && P.gc.bound[c] == ch.p0, "list-major chunk order");
      ga.item_off = b.chunk_items + c;
      ga.item_counter = b.counter + 1 + c;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        e0 = newev();
        e1 = newev();
        tr.scan.push_back(e0);
        tr.scan.push_back(e1);
        RBQ_HIP(hipEventRecord(e0, s));
      }
      if (P.flat) {
        FlatArgs fl;
        fl.blocks = idx->flat.as<float>();
        fl.pos2id = idx->pos2id.as<int32_t>();
        fl.d = d;
        fl.q = qd;
        fl.ldq = need_qcopy ? ld : d;
        fl.nq = (int)nq;
        fl.nprobe = nprobe;
        fl.R = R;
        fl.G = P.G;
        fl.slots = ga.slots;
        fl.item_off = ga.item_off;
        fl.items = ga.items;
        fl.item_counter = ga.item_counter;
        fl.qthr = ga.qthr;
        fl.pool = ga.pool;
        fl.pool_ld = ga.pool_ld;
        fl.cap = ga.cap;
        fl.pcnt = ga.pcnt;
        fl.overflow = ga.overflow;
        fl.any_overflow = ga.any_overflow;
        launch_scan_flat(s, fl, P.wg_per_cu * idx->num_cus);
      } else {
        launch_scan_group(s, ga, P.wg_per_cu * idx->num_cus);
      }
      if (timed) {
        RBQ_HIP(hipEventRecord(e1, s));
        tr.scan_lm.push_back(1);
        tr.group += 1;
        unsigned long long* tc = idx->tcounter.as<unsigned long long>();
        for (int part = 0; part < 2; ++part) {  // all scans, and list-major alone
          hipLaunchKernelGGL(k_count_scanned, dim3(64), dim3(256), 0, s, b.probes,
                             idx->list_len.as<int32_t>(), (int)nq, nprobe, ch.p0, ch.pn, rec_bytes, 0,
                             tc + 2 * part);
          hipLaunchKernelGGL(k_count_group_bytes, dim3(16), dim3(256), 0, s, b.gcnt + (int64_t)c * nlist,
                             idx->list_len.as<int32_t>(), nlist, ga.G, rec_bytes, tc + 2 * part + 1);
        }
        RBQ_HIP(hipGetLastError());
      }
      ma.max_extra = (int)pool_cap;
      // (the first list-major chunk's pools, filled before any threshold,
      // are the long rows; later ones mostly fit one 256-thread piece)
      ma.merge_threads = (P.merge == 2 || (P.merge == 1 && c > 0)) ? 256 : 512;
      launch_row_topk(s, ma, (int)nq);
    };
    FusedArgs fa;
    fa.L = sa.L;
    fa.Q = sa.Q;
    fa.probes = b.probes;
    fa.nq = (int)nq;
    fa.nprobe = nprobe;
    fa.R = R;
    fa.out = b.cand;
    fa.out_ld = cand_ld;
    fa.qthr = b.qthr;
    fa.rowk = d_R;
    fa.qmask = nullptr;
    auto scan_fused_chunk = [&](const Chunk& ch) {
      fa.p0 = ch.p0;
      fa.pn = ch.pn;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (timed) {
        e0 = newev();
        e1 = newev();
        tr.scan.push_back(e0);
        tr.scan.push_back(e1);
        RBQ_HIP(hipEventRecord(e0, s));
      }
      launch_scan_fused(s, fa);  // scan and selection in one launch: no merge
      if (timed) {
        RBQ_HIP(hipEventRecord(e1, s));
        tr.scan_lm.push_back(2);
        tr.popc += 1;
        tr.fused += 1;
        unsigned long long* tc = idx->tcounter.as<unsigned long long>();
        for (int slot : {0, 4})  // all scans, and the fused ones alone
          hipLaunchKernelGGL(k_count_scanned, dim3(64), dim3(256), 0, s, b.probes,
                             idx->list_len.as<int32_t>(), (int)nq, nprobe, ch.p0, ch.pn, rec_bytes, 1,
                             tc + slot);
        RBQ_HIP(hipGetLastError());
      }
    };
    for (const auto& ch : chunks) {
      if (ch.lm)
        scan_group_chunk(ch);
      else if (ch.fused)
        scan_fused_chunk(ch);
      else
        scan_popc_chunk(ch);
    }
    // Queries whose pool overflowed in a list-major chunk are searched again,
    // from scratch and exactly. On the device (d <= 1024): the fused scan,
    // masked to them, starts each afresh (empty running top-R, no threshold)
    // and covers every probe rank; its workgroups of other queries return at
    // once, so nothing waits for the host. Otherwise their rows are reset and
    // the host reads one flag and, if it is set, the query-major scan redoes
    // them.
    if (any_group && P.flat) {
      // IVF-Flat has no second scan form to redo a query with: a pool that
      // overflowed fails the search rather than returning a wrong result
      uint32_t any = 0;
      RBQ_HIP(hipMemcpyAsync(&any, b.counter, sizeof(any), hipMemcpyDeviceToHost, s));
      RBQ_HIP(hipStreamSynchronize(s));
      if (any)
        fail(RBQ_ENOMEM, "IVF-Flat: a query's candidate pool overflowed; search fewer queries per batch");
    } else if (any_group) {
      if (idx->W <= 32) {
        FusedArgs ra = fa;
        ra.p0 = 0;
        ra.pn = nprobe;
        ra.qmask = b.overflow;
        ra.reset = 1;
        launch_scan_fused(s, ra);
        if (timed) {
          hipLaunchKernelGGL(k_count_flags, dim3(16), dim3(256), 0, s, b.overflow, (int)nq,
                             idx->tcounter.as<unsigned long long>() + 6);
          RBQ_HIP(hipGetLastError());
        }
      } else {
        launch_reset_masked(s, b.overflow, b.cand, cand_ld, R, b.qthr, b.pcnt, (int)nq);
        uint32_t any = 0;
        RBQ_HIP(hipMemcpyAsync(&any, b.counter, sizeof(any), hipMemcpyDeviceToHost, s));
        RBQ_HIP(hipStreamSynchronize(s));
        if (any) {
          sa.qmask = b.overflow;
          for (const auto& ch : qm_chunks) scan_popc_chunk(ch);
          sa.qmask = nullptr;
        }
      }
    }
    int64_t* ids_out = ids_dev ? ids : b.ids;
    float* dist_out = dist_dev ? dist : b.dist;
    const uint64_t* top = b.cand;
    if (dbg && (dbg->cand_ids || dbg->cand_est)) {  // the debug output lists candidates ascending
      TopkArgs so;
      so.keys = b.cand;
      so.ld = cand_ld;
      so.ncols = R;
      so.k = R;
      so.out_keys = b.cand;
      so.ldo = cand_ld;
      so.rowk = d_R;
      launch_row_topk(s, so, (int)nq);
    }
    mark(4);
    hipStream_t release_on = s;  // the stream whose last use of the workspace ends it
    if (job) {
      // Phase 5 on host cores: hand the candidates (and the queries, if they
      // are only on the device) over in pinned memory, on the job's copy
      // stream when it has one (not with debug outputs, which read the
      // workspace on this stream afterwards)
      hipStream_t cs = s;
      if (job->copy && !dbg) {
        RBQ_HIP(hipEventRecord(job->staged, s));
        RBQ_HIP(hipStreamWaitEvent(job->copy, job->staged, 0));
        cs = release_on = job->copy;
      }
      RBQ_HIP(hipMemcpy2DAsync(job->cand, R * sizeof(uint64_t), top, cand_ld * sizeof(uint64_t),
                               R * sizeof(uint64_t), nq, hipMemcpyDeviceToHost, cs));
      if (qdev)
        RBQ_HIP(hipMemcpy2DAsync(job->qh, d * sizeof(float), qd, (need_qcopy ? ld : d) * sizeof(float),
                                 d * sizeof(float), nq, hipMemcpyDeviceToHost, cs));
      RBQ_HIP(hipEventRecord(job->ready, cs));
    } else {
      // Phase 5: exact re-rank of the top-R on the GPU
      if (idx->X8.p)
        launch_rerank_u8(s, qd, ld, idx->X8.as<uint8_t>(), idx->n, ld, d, top, cand_ld, (int)nq, R, k,
                         ids_out, dist_out, d_k);
      else
        launch_rerank(s, qd, ld, idx->X.as<float>(), idx->n, ld, d, top, cand_ld, (int)nq, R, k,
                      ids_out, dist_out, d_k);
    }
    if (timed) RBQ_HIP(hipEventRecord(tr.e[5], release_on));

    // host-side outputs
    if (ids && !ids_dev)
      RBQ_HIP(hipMemcpyAsync(ids, b.ids, (size_t)nq * k * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if (dist && !dist_dev)
      RBQ_HIP(hipMemcpyAsync(dist, b.dist, (size_t)nq * k * sizeof(float), hipMemcpyDeviceToHost, s));
    std::vector<uint64_t> hm;
    if (dbg) {
      if (dbg->probes)
        RBQ_HIP(hipMemcpyAsync(dbg->probes, b.probes, pairs * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      if (dbg->probe_score && b.pscore)
        RBQ_HIP(hipMemcpyAsync(dbg->probe_score, b.pscore, pairs * sizeof(float), hipMemcpyDeviceToHost, s));
      if (dbg->qrot)
        RBQ_HIP(hipMemcpy2DAsync(dbg->qrot, d * sizeof(float), b.qrot, ld * sizeof(float),
                                 d * sizeof(float), nq, hipMemcpyDeviceToHost, s));
      if (dbg->qu && !P.unq)
        RBQ_HIP(hipMemcpy2DAsync(dbg->qu, d, b.qu, W * 32, d, pairs, hipMemcpyDeviceToHost, s));
      if (dbg->scalars && !P.unq)
        RBQ_HIP(hipMemcpyAsync(dbg->scalars, b.scal, pairs * sizeof(float4), hipMemcpyDeviceToHost, s));
      if (dbg->ip)
        RBQ_HIP(hipMemcpyAsync(dbg->ip, b.dump_ip, (size_t)pairs * maxlen * sizeof(int32_t),
                               hipMemcpyDeviceToHost, s));
      if (dbg->est)
        RBQ_HIP(hipMemcpyAsync(dbg->est, b.dump_est, (size_t)pairs * maxlen * sizeof(float),
                               hipMemcpyDeviceToHost, s));
      if (dbg->cand_ids || dbg->cand_est) {
        hm.resize((size_t)nq * R);
        RBQ_HIP(hipMemcpy2DAsync(hm.data(), R * sizeof(uint64_t), top, cand_ld * sizeof(uint64_t),
                                 R * sizeof(uint64_t), nq, hipMemcpyDeviceToHost, s));
      }
      if (dbg->ids && !job)
        RBQ_HIP(hipMemcpyAsync(dbg->ids, ids_out, (size_t)nq * k * sizeof(int64_t),
                               hipMemcpyDeviceToHost, s));
      if (dbg->sqdist && !job)
        RBQ_HIP(hipMemcpyAsync(dbg->sqdist, dist_out, (size_t)nq * k * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    if (ws) ws_release(idx, std::move(ws), release_on);
    if (timed) {
      tr.first_part = !io.continues_search;
      std::lock_guard<std::mutex> g(idx->timing_mu);
      idx->pending.push_back(std::move(tr));
    }
    const bool host_out = (ids && !ids_dev) || (dist && !dist_dev) || dbg;
    if (host_out) RBQ_HIP(hipStreamSynchronize(s));
    if (dbg && !hm.empty()) {
      for (size_t t = 0; t < hm.size(); ++t) {
        const uint64_t v = hm[t];
        if (dbg->cand_ids) dbg->cand_ids[t] = v == KEY_NONE ? -1 : (int64_t)(uint32_t)v;
        if (dbg->cand_est) dbg->cand_est[t] = v == KEY_NONE ? INFINITY : f32_ord((uint32_t)(v >> 32));
      }
    }
  }
}

ThreadPool& host_pool(rbq_index* idx) {
  std::lock_guard<std::mutex> g(idx->host_mu);
  if (!idx->pool) {
    int t = idx->host_threads;
    // automatic: up to 16, less two when there are 8 or more: the threads
    // that queue GPU work must not wait for a core (a queue left idle stalls
    // the GPU), nor may the process exceed its share of the host
    if (t <= 0) {
      t = (int)std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
      if (t >= 8) t -= 2;
    }
    idx->pool.reset(new ThreadPool(t));
  }
  return *idx->pool;
}

// Search with the re-rank on host cores (raw vectors in host memory).
// The batch is cut into sub-batches: while the host threads re-rank one, the
// GPU already searches the next (the overlap of Sec. 3.3.4).
void search_host_rerank(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R,
                        int64_t* ids, float* dist, hipStream_t s, const SearchIO& io) {
  const int d = idx->d;
  const bool qdev = is_device_ptr(q);
  const bool ids_dev = ids && is_device_ptr(ids), dist_dev = dist && is_device_ptr(dist);
  const rbq_debug_io* dbg = io.dbg;
  const int parts = dbg ? 1 : host_rerank_parts(idx, nq, nprobe);
  const int64_t sb = ceil_div(nq, (int64_t)parts);
  const bool stage_out = !ids || !dist || ids_dev || dist_dev;
  size_t off = 0;
  auto carve = [&](size_t bytes) {
    const size_t o = off;
    off = (off + bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_cand = carve((size_t)nq * R * sizeof(uint64_t));
  const size_t o_q = qdev ? carve((size_t)nq * d * sizeof(float)) : 0;
  const size_t o_ids = stage_out ? carve((size_t)nq * k * sizeof(int64_t)) : 0;
  const size_t o_dist = stage_out ? carve((size_t)nq * k * sizeof(float)) : 0;
  Pinned pin(idx, std::max<size_t>(off, 256));
  char* base = static_cast<char*>(pin.p);
  uint64_t* hc = reinterpret_cast<uint64_t*>(base + o_cand);
  float* hq = qdev ? reinterpret_cast<float*>(base + o_q) : const_cast<float*>(q);
  int64_t* hids = stage_out ? reinterpret_cast<int64_t*>(base + o_ids) : ids;
  float* hdist = stage_out ? reinterpret_cast<float*>(base + o_dist) : dist;

  ThreadPool& pool = host_pool(idx);
  Latch latch;
  std::mutex emu;
  std::string err;
  rbq_status est = RBQ_OK;
  std::vector<hipEvent_t> events, staged;
  auto wait_all = [&]() {
    latch.wait();
    for (hipEvent_t e : events) (void)hipEventDestroy(e);
    for (hipEvent_t e : staged) (void)hipEventDestroy(e);
    events.clear();
    staged.clear();
  };
  hipStream_t gs = nullptr, cs = nullptr;
  {
    std::lock_guard<std::mutex> g(idx->host_mu);
    if (!idx->host_gpu_stream) RBQ_HIP(hipStreamCreateWithFlags(&idx->host_gpu_stream, hipStreamNonBlocking));
    if (!idx->host_copy_stream) RBQ_HIP(hipStreamCreateWithFlags(&idx->host_copy_stream, hipStreamNonBlocking));
    gs = idx->host_gpu_stream;
    cs = idx->host_copy_stream;
  }
  hipEvent_t inputs = nullptr;  // the caller's stream has its queries ready
  RBQ_HIP(hipEventCreateWithFlags(&inputs, hipEventDisableTiming));
  events.push_back(inputs);
  RBQ_HIP(hipEventRecord(inputs, s));
  try {
    // every sub-batch's GPU work is queued first, on the index's host-path
    // stream and as one block; then, as each completes (the caller sleeps on
    // its event rather than spinning), its re-rank goes to the host threads,
    // so they only ever hold work that is ready
    std::vector<std::pair<int64_t, int64_t>> ranges;
    std::unique_lock<std::mutex> enqueue(idx->host_gpu_mu);
    RBQ_HIP(hipStreamWaitEvent(gs, inputs, 0));
    for (int64_t q0 = 0; q0 < nq; q0 += sb) {
      const int64_t q1 = std::min(nq, q0 + sb);
      HostJob job;
      job.cand = hc + q0 * R;
      job.qh = hq + q0 * d;
      RBQ_HIP(hipEventCreateWithFlags(&job.ready, hipEventDisableTiming | hipEventBlockingSync));
      events.push_back(job.ready);
      RBQ_HIP(hipEventCreateWithFlags(&job.staged, hipEventDisableTiming));
      staged.push_back(job.staged);
      job.copy = cs;
      ranges.emplace_back(q0, q1);
      SearchIO sub = io;
      sub.continues_search = q0 > 0;
      if (io.q_nprobe) {
        sub.q_nprobe = io.q_nprobe + q0;
        sub.q_k = io.q_k + q0;
        sub.q_R = io.q_R + q0;
      }
      const float* qsrc = q + q0 * d;
      search_part(idx, qsrc, q1 - q0, nprobe, k, R, nullptr, nullptr, gs, sub, &job);
    }
    enqueue.unlock();
    for (size_t pi = 0; pi < ranges.size(); ++pi) {
      RBQ_HIP(hipEventSynchronize(events[pi + 1]));
      const int64_t q0 = ranges[pi].first, q1 = ranges[pi].second;
      const int tasks = std::max(1, std::min<int>(pool.size(), (int)ceil_div(q1 - q0, (int64_t)8)));
      const int64_t per = ceil_div(q1 - q0, (int64_t)tasks);
      for (int64_t r0 = q0; r0 < q1; r0 += per) {
        const int64_t r1 = std::min(q1, r0 + per);
        latch.add(1);
        pool.submit([=, &latch, &emu, &err, &est]() {
          try {
            host_rerank_rows(idx->hostX, idx->n, d, hq, hc, R, io.q_k, k, r0, r1, hids, hdist);
          } catch (const Error& e) {
            std::lock_guard<std::mutex> g(emu);
            est = e.status;
            err = e.what();
          } catch (const std::exception& e) {
            std::lock_guard<std::mutex> g(emu);
            est = RBQ_EDEVICE;
            err = e.what();
          }
          latch.done();
        });
      }
    }
  } catch (...) {
    (void)hipStreamSynchronize(gs);
    (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(s);
    wait_all();
    throw;
  }
  wait_all();
  if (est != RBQ_OK) throw Error(est, err);
  if (ids && ids != hids)
    RBQ_HIP(hipMemcpyAsync(ids, hids, (size_t)nq * k * sizeof(int64_t), hipMemcpyDefault, s));
  if (dist && dist != hdist)
    RBQ_HIP(hipMemcpyAsync(dist, hdist, (size_t)nq * k * sizeof(float), hipMemcpyDefault, s));
  if (dbg && dbg->ids) std::memcpy(dbg->ids, hids, (size_t)nq * k * sizeof(int64_t));
  if (dbg && dbg->sqdist) std::memcpy(dbg->sqdist, hdist, (size_t)nq * k * sizeof(float));
  RBQ_HIP(hipStreamSynchronize(s));  // the staging is reused once the copies are done
}

}  // namespace

// Sub-batches of a host re-rank search: more of them overlap more of the
// host's work with the GPU's, but each list-major item then groups fewer
// queries, so the automatic rule keeps at least 8 (query, list) pairs per
// list in each sub-batch on average.
int host_rerank_parts(const rbq_index* idx, int64_t nq, int nprobe) {
  const int fixed = idx->opt_host_parts.load();
  if (fixed > 0) return (int)std::min<int64_t>(fixed, std::max<int64_t>(1, nq));
  int parts = nq >= 2048 ? 4 : (nq >= 256 ? 2 : 1);
  while (parts > 1 && nq * (int64_t)nprobe < (int64_t)8 * parts * idx->nlist) parts /= 2;
  return parts;
}

void search_candidates(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R,
                       uint64_t* cand_host, float* q_host, hipStream_t s, const SearchIO& io) {
  if (nq == 0) return;
  RBQ_HIP(hipSetDevice(idx->device));
  HostJob job;
  job.cand = cand_host;
  job.qh = q_host;
  RBQ_HIP(hipEventCreateWithFlags(&job.ready, hipEventDisableTiming));
  try {
    search_part(idx, q, nq, nprobe, k, R, nullptr, nullptr, s, io, &job);
    RBQ_HIP(hipEventSynchronize(job.ready));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(job.ready);
    throw;
  }
  RBQ_HIP(hipEventDestroy(job.ready));
}

void search(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R, int64_t* ids,
            float* dist, hipStream_t s, const SearchIO& io) {
  if (nq == 0) return;
  if (idx->vectors_on_host) {
    RBQ_HIP(hipSetDevice(idx->device));
    search_host_rerank(idx, q, nq, nprobe, k, R, ids, dist, s, io);
  } else {
    search_part(idx, q, nq, nprobe, k, R, ids, dist, s, io, nullptr);
  }
}

}  // namespace rbq
