// Autotuner: measures the launch choices of a search that leave its results
// unchanged (scan form, queries per list-major item, persistent grid size,
// first chunk size) for one batch shape, and keeps the fastest per bucket of
// (nq, nprobe, rerank_n) rounded up to powers of two. Every later search whose
// shape falls in a tuned bucket uses the stored choices. The table can be saved
// to and loaded from a text cache, whose entries are keyed by a signature of
// the device architecture, D, B_q, nlist, n and the list-size histogram.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

#include "index.hpp"

namespace rbq {

namespace {

int ceil_log2(int64_t v) {
  int b = 0;
  while ((int64_t(1) << b) < v) ++b;
  return b;
}

std::string signature(const rbq_index* idx) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, idx->device) == hipSuccess) {
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
  } else {
    (void)hipGetLastError();
  }
  // list sizes by power-of-two bucket, hashed (FNV-1a)
  uint32_t hist[33] = {};
  for (int32_t len : idx->h_list_len) hist[ceil_log2((int64_t)len + 1)] += 1;
  uint64_t h = 1469598103934665603ull;
  for (uint32_t c : hist)
    for (int b = 0; b < 4; ++b) {
      h ^= (c >> (8 * b)) & 0xFFu;
      h *= 1099511628211ull;
    }
  char buf[256];
  std::snprintf(buf, sizeof(buf), "%s:d=%d:bq=%d:nlist=%d:n=%lld:hist=%016llx", arch.c_str(), idx->d,
                idx->bq, idx->nlist, (long long)idx->n, (unsigned long long)h);
  return buf;
}

}  // namespace

uint64_t tune_key(int64_t nq, int nprobe, int R) {
  return ((uint64_t)ceil_log2(nq) << 16) | ((uint64_t)ceil_log2(nprobe) << 8) | (uint64_t)ceil_log2(R);
}

bool tune_lookup(rbq_index* idx, int64_t nq, int nprobe, int R, TuneCfg* out) {
  std::lock_guard<std::mutex> g(idx->tune_mu);
  if (idx->tune.empty()) return false;
  const auto it = idx->tune.find(tune_key(nq, nprobe, R));
  if (it == idx->tune.end()) return false;
  *out = it->second;
  return true;
}

void autotune(rbq_index* idx, const float* q, int64_t nq, int nprobe, int k, int R,
              rbq_tune_result* out) {
  RBQ_HIP(hipSetDevice(idx->device));
  // With the re-rank on host cores a search runs on the GPU in sub-batches:
  // the choices are tuned, and stored, for the sub-batch (its first queries)
  if (idx->vectors_on_host) nq = ceil_div(nq, (int64_t)host_rerank_parts(idx, nq, nprobe));
  const int d = idx->d;
  std::vector<TuneCfg> cands;
  cands.push_back(TuneCfg{1, 64, 8, 2, 4, 2, 0});
  if (group_k_steps(d) <= 4)
    for (int gm : {0, 4, 16, 64})
      for (int early : {0, 1}) {
        // (gm 0: every chunk list-major, no early chunks; gm 64: early only
        // for the batch shapes where list-major rarely pays, fused kept)
        if (early == 1 && (gm == 0 || gm == 64)) continue;
        for (int G : {32, 64})
          for (int wg : {4, 8})
            for (int ff : {1, 2, 4})
              for (int gr : {2, 3, 4, 6, 8}) cands.push_back(TuneCfg{2, G, wg, ff, gm, gr, early});
      }

  hipStream_t s = nullptr;
  RBQ_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const int saved_timing = idx->timing.exchange(0);
  DevBuf dq, ids, dist;
  try {
    RBQ_HIP(hipEventCreate(&e0));
    RBQ_HIP(hipEventCreate(&e1));
    dq.alloc((size_t)nq * d * sizeof(float));
    RBQ_HIP(hipMemcpyAsync(dq.p, q, (size_t)nq * d * sizeof(float), hipMemcpyDefault, s));
    ids.alloc((size_t)nq * k * sizeof(int64_t));
    dist.alloc((size_t)nq * k * sizeof(float));
    std::vector<int64_t> ref_ids((size_t)nq * k), got_ids((size_t)nq * k);
    std::vector<float> ref_d((size_t)nq * k), got_d((size_t)nq * k);
    {  // the built-in rule for this shape (no table entry while it is timed)
      std::lock_guard<std::mutex> g(idx->tune_mu);
      idx->tune.erase(tune_key(nq, nprobe, R));
    }
    // With the raw vectors on the host the re-rank runs on host cores and no
    // launch choice touches it: the choices are timed on the GPU phases alone
    // (probe to coarse top-R) and compared on the candidates they return.
    const bool host_rr = idx->vectors_on_host != 0;
    uint64_t* hc = nullptr;
    float* hq = nullptr;
    std::vector<uint64_t> ref_c, got_c;
    if (host_rr) {
      RBQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&hc), (size_t)nq * R * sizeof(uint64_t), hipHostMallocDefault));
      RBQ_HIP(hipHostMalloc(reinterpret_cast<void**>(&hq), (size_t)nq * d * sizeof(float), hipHostMallocDefault));
      ref_c.resize((size_t)nq * R);
      got_c.resize((size_t)nq * R);
    }
    struct PinnedFree {
      void* a;
      void* b;
      ~PinnedFree() {
        if (a) (void)hipHostFree(a);
        if (b) (void)hipHostFree(b);
      }
    } pinned_guard{hc, hq};
    // Each choice is timed over three searches, or over one when that one
    // already takes over 1.5x the best time so far (it cannot win).
    float best_ms = 0.f;
    auto time_cfg = [&](const TuneCfg* cfg, std::vector<int64_t>& oi, std::vector<float>& od) {
      SearchIO io;
      io.force = cfg;
      constexpr int reps = 3;
      if (host_rr) {
        std::vector<uint64_t>& oc = &oi == &ref_ids ? ref_c : got_c;
        search_candidates(idx, dq.as<float>(), nq, nprobe, k, R, hc, hq, s, io);
        std::memcpy(oc.data(), hc, oc.size() * sizeof(uint64_t));
        // (a query's candidates come in no particular order: compare them
        // sorted; rows sorted on several host threads)
        const int64_t nt = std::min<int64_t>(16, std::max<int64_t>(1, nq / 64));
        std::vector<std::thread> th;
        for (int64_t t = 0; t < nt; ++t)
          th.emplace_back([&, t] {
            for (int64_t i = t * nq / nt; i < (t + 1) * nq / nt; ++i)
              std::sort(oc.begin() + i * R, oc.begin() + (i + 1) * R);
          });
        for (auto& x : th) x.join();
        float total = 0.f;
        for (int r = 0; r < reps; ++r) {
          const auto t0 = std::chrono::steady_clock::now();
          search_candidates(idx, dq.as<float>(), nq, nprobe, k, R, hc, hq, s, io);
          total += std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - t0).count();
          if (r == 0 && best_ms > 0.f && total > 1.5f * best_ms) return total;
        }
        return total / reps;
      }
      search(idx, dq.as<float>(), nq, nprobe, k, R, ids.as<int64_t>(), dist.as<float>(), s, io);
      RBQ_HIP(hipMemcpyAsync(oi.data(), ids.p, oi.size() * sizeof(int64_t), hipMemcpyDeviceToHost, s));
      RBQ_HIP(hipMemcpyAsync(od.data(), dist.p, od.size() * sizeof(float), hipMemcpyDeviceToHost, s));
      float total = 0.f;
      for (int r = 0; r < reps; ++r) {
        RBQ_HIP(hipEventRecord(e0, s));
        search(idx, dq.as<float>(), nq, nprobe, k, R, ids.as<int64_t>(), dist.as<float>(), s, io);
        RBQ_HIP(hipEventRecord(e1, s));
        RBQ_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        RBQ_HIP(hipEventElapsedTime(&ms, e0, e1));
        total += ms;
        if (r == 0 && best_ms > 0.f && total > 1.5f * best_ms) return total;
      }
      return total / reps;
    };
    const float ms_default = time_cfg(nullptr, ref_ids, ref_d);
    TuneCfg best;
    bool have = false;
    for (const TuneCfg& c : cands) {
      const float ms = time_cfg(&c, got_ids, got_d);
      // every choice computes the same exact selection
      const bool differs = host_rr ? got_c != ref_c
                                   : (got_ids != ref_ids ||
                                      std::memcmp(got_d.data(), ref_d.data(), got_d.size() * 4) != 0);
      if (differs) {
        char msg[192];
        std::snprintf(msg, sizeof(msg),
                      "autotune: launch choices returned different results (scan %d G %d wg_per_cu %d "
                      "first_factor %d gm %d growth %d early %d)",
                      c.scan, c.G, c.wg_per_cu, c.first_factor, c.gm, c.growth, c.early);
        fail(RBQ_EDEVICE, msg);
      }
      if (!have || ms < best_ms) {
        best = c;
        best_ms = ms;
        have = true;
      }
    }
    // then the index-block size of the best list-major choice (Sec. 3.3.1:
    // long lists shared out over several workgroups), results checked alike
    int trials = (int)cands.size();
    if (best.scan == 2) {
      const TuneCfg base = best;
      for (int B : {8, 16, 32, 64}) {
        TuneCfg c = base;
        c.B = B;
        const float ms = time_cfg(&c, got_ids, got_d);
        ++trials;
        const bool differs = host_rr ? got_c != ref_c
                                     : (got_ids != ref_ids ||
                                        std::memcmp(got_d.data(), ref_d.data(), got_d.size() * 4) != 0);
        if (differs) fail(RBQ_EDEVICE, "autotune: index blocks of " + std::to_string(B) +
                                           " micro-blocks returned different results");
        if (ms < best_ms) {
          best = c;
          best_ms = ms;
        }
      }
    }
    // then which pool merges run on 256-thread workgroups
    {
      const TuneCfg base = best;
      for (int mg : {1, 2}) {
        TuneCfg c = base;
        c.merge = mg;
        const float ms = time_cfg(&c, got_ids, got_d);
        ++trials;
        const bool differs = host_rr ? got_c != ref_c
                                     : (got_ids != ref_ids ||
                                        std::memcmp(got_d.data(), ref_d.data(), got_d.size() * 4) != 0);
        if (differs) fail(RBQ_EDEVICE, "autotune: 256-thread pool merges returned different results");
        if (ms < best_ms) {
          best = c;
          best_ms = ms;
        }
      }
    }
    {
      std::lock_guard<std::mutex> g(idx->tune_mu);
      idx->tune[tune_key(nq, nprobe, R)] = best;
    }
    if (out) {
      std::memset(out, 0, sizeof(*out));
      out->scan = best.scan;
      out->group_size = best.G;
      out->wg_per_cu = best.wg_per_cu;
      out->first_factor = best.first_factor;
      out->chunk_group_min = best.gm;
      out->growth = best.growth;
      out->early_form = best.early;
      out->block = best.B;
      out->merge_form = best.merge;
      out->ms = best_ms;
      out->ms_default = ms_default;
      out->trials = (int32_t)trials;
    }
  } catch (...) {
    (void)hipStreamSynchronize(s);
    idx->timing.store(saved_timing);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    throw;
  }
  idx->timing.store(saved_timing);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  RBQ_HIP(hipStreamSynchronize(s));
  RBQ_HIP(hipStreamDestroy(s));
}

// Cache file: one entry per line,
// "<signature> <key> <scan> <G> <wg> <ff> <gm> <growth> <early>";
// lines of other signatures are kept when this index's entries are rewritten.
void tune_save(rbq_index* idx, const char* path) {
  const std::string sig = signature(idx);
  std::vector<std::string> keep;
  {
    std::ifstream in(path);
    std::string line;
    while (std::getline(in, line))
      if (!line.empty() && line[0] != '#' && line.compare(0, sig.size() + 1, sig + " ") != 0)
        keep.push_back(line);
  }
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    RBQ_CHECK(o.good(), "cannot write the autotune cache");
    o << "# librbq autotune cache v6: signature key scan G wg_per_cu first_factor gm growth early block merge\n";
    for (const auto& l : keep) o << l << "\n";
    std::lock_guard<std::mutex> g(idx->tune_mu);
    for (const auto& kv : idx->tune)
      o << sig << " " << kv.first << " " << kv.second.scan << " " << kv.second.G << " "
        << kv.second.wg_per_cu << " " << kv.second.first_factor << " " << kv.second.gm << " "
        << kv.second.growth << " " << kv.second.early << " " << kv.second.B << " " << kv.second.merge << "\n";
    RBQ_CHECK(o.good(), "writing the autotune cache failed");
  }
  RBQ_CHECK(std::rename(tmp.c_str(), path) == 0, "cannot replace the autotune cache");
}

int tune_load(rbq_index* idx, const char* path) {
  std::ifstream in(path);
  RBQ_CHECK(in.good(), "cannot read the autotune cache");
  const std::string sig = signature(idx);
  std::string line;
  int loaded = 0;
  std::map<uint64_t, TuneCfg> got;
  while (std::getline(in, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream ls(line);
    std::string s;
    uint64_t key = 0;
    TuneCfg c;
    if (!(ls >> s >> key >> c.scan >> c.G >> c.wg_per_cu >> c.first_factor >> c.gm >> c.growth >> c.early >>
          c.B >> c.merge))
      continue;
    if (s != sig) continue;
    const bool ok = (c.scan == 1 || c.scan == 2) && c.G >= 1 && c.G <= 64 && c.wg_per_cu >= 1 &&
                    c.wg_per_cu <= 64 && c.first_factor >= 1 && c.first_factor <= 64 &&
                    c.gm >= 0 && c.gm <= (1 << 20) && c.growth >= 2 && c.growth <= 16 &&
                    (c.early == 0 || c.early == 1) && c.B >= 0 && c.B <= (1 << 20) && c.merge >= 0 &&
                    c.merge <= 2;
    RBQ_CHECK(ok, "autotune cache entry out of range");
    got[key] = c;
    ++loaded;
  }
  std::lock_guard<std::mutex> g(idx->tune_mu);
  for (const auto& kv : got) idx->tune[kv.first] = kv.second;
  return loaded;
}

}  // namespace rbq
