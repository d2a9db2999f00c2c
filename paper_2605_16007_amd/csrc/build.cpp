// Index construction (Sec. 3.1.1): k-means centroids (Phases 1-2: random
// k-means++ seeding, GPU assignment, host centroid update), assignment of every
// vector, random orthogonal P, list layout, and the RaBitQ encoding (Phase 3).
#include <sys/mman.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <thread>

#include "host_math.hpp"
#include "index.hpp"

namespace rbq {

namespace {
// Progress on stderr when the environment sets RBQ_LOG to a value other than
// 0 (a 400M-row build runs for minutes inside one call; workspace sizes).
bool build_log_on() {
  static const bool on = [] {
    const char* v = std::getenv("RBQ_LOG");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void build_log(const char* fmt, ...) {
  if (!build_log_on()) return;
  static const auto t0 = std::chrono::steady_clock::now();
  const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  char msg[256];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[rbq %8.1fs] %s\n", t, msg);
  std::fflush(stderr);
}

}  // namespace

Workspace::~Workspace() {
  if (done) (void)hipEventDestroy(done);
  if (base) (void)hipFree(base);
}

void DevBuf::alloc(size_t b) {
  reset();
  if (b == 0) b = 256;
  RBQ_HIP(hipMalloc(&p, b));
  bytes = b;
}

void DevBuf::reset() {
  if (p) {
    (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
}

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

// The host re-rank gathers one random row per candidate, so its rate is set by
// TLB reach more than by bandwidth: the rows live in anonymous memory aligned
// to and advised for 2 MiB transparent huge pages. Only host threads read
// them, so they are not pinned (pinned pages stay 4 KiB).
constexpr size_t kHugePage = size_t(2) << 20;

float* host_rows_alloc(size_t bytes, size_t* mapped) {
  const size_t len = (std::max<size_t>(bytes, 1) + kHugePage - 1) / kHugePage * kHugePage;
  void* raw = mmap(nullptr, len + kHugePage, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
  if (raw == MAP_FAILED) fail(RBQ_ENOMEM, "host rows: mmap of " + std::to_string(len) + " bytes failed");
  const uintptr_t b = reinterpret_cast<uintptr_t>(raw);
  const uintptr_t a = (b + kHugePage - 1) & ~(uintptr_t)(kHugePage - 1);
  if (a > b) munmap(raw, a - b);  // trim to a 2 MiB-aligned range of len bytes
  if (a + len < b + len + kHugePage) munmap(reinterpret_cast<void*>(a + len), b + kHugePage - a);
  (void)madvise(reinterpret_cast<void*>(a), len, MADV_HUGEPAGE);  // advice only
  *mapped = len;
  return reinterpret_cast<float*>(a);
}

void host_rows_free(float* p, size_t mapped) {
  if (p && mapped) munmap(p, mapped);
}

void host_rows_fill(float* dst, const float* src, size_t count, int threads) {
  const size_t nt = (size_t)std::max(1, threads);
  const size_t per = std::max<size_t>(1 << 20, (count + nt - 1) / nt);
  std::vector<std::thread> ts;
  for (size_t o = 0; o < count; o += per) {
    const size_t m = std::min(per, count - o);
    ts.emplace_back([=] { std::memcpy(dst + o, src + o, m * sizeof(float)); });
  }
  for (auto& t : ts) t.join();
}

// Searches enqueue their work and hand their workspace back at once, so a
// caller that issues searches faster than the GPU completes them would keep
// allocating: once kMaxIdleWorkspaces are held back, the oldest one is waited
// for and reused instead.
constexpr size_t kMaxIdleWorkspaces = 4;

std::unique_ptr<Workspace> ws_acquire(rbq_index* idx, size_t bytes) {
  std::unique_ptr<Workspace> got;
  bool wait = false;
  {
    std::lock_guard<std::mutex> g(idx->ws_mu);
    // prefer the smallest idle workspace that is big enough
    size_t best = (size_t)-1;
    for (size_t i = 0; i < idx->ws_free.size(); ++i) {
      auto& w = idx->ws_free[i];
      if (hipEventQuery(w->done) != hipSuccess) {
        (void)hipGetLastError();
        continue;
      }
      if (w->cap >= bytes && (best == (size_t)-1 || w->cap < idx->ws_free[best]->cap)) best = i;
    }
    if (best == (size_t)-1) {
      for (size_t i = 0; i < idx->ws_free.size(); ++i)
        if (hipEventQuery(idx->ws_free[i]->done) == hipSuccess) {
          best = i;
          break;
        }
      (void)hipGetLastError();
    }
    if (best == (size_t)-1 && idx->ws_free.size() >= kMaxIdleWorkspaces) {
      best = 0;  // every held workspace is still in use: the oldest
      wait = true;
    }
    if (best != (size_t)-1) {
      got = std::move(idx->ws_free[best]);
      idx->ws_free.erase(idx->ws_free.begin() + best);
    }
  }
  if (wait) RBQ_HIP(hipEventSynchronize(got->done));
  if (got && got->cap >= bytes) return got;
  got.reset();  // idle but too small: its last use has completed
  build_log("search workspace: allocating %.3f GB", (double)bytes / 1e9);
  got = std::make_unique<Workspace>();
  RBQ_HIP(hipMalloc(reinterpret_cast<void**>(&got->base), bytes));
  got->cap = bytes;
  // (blocking: a search that must wait for a workspace sleeps, leaving the
  // host cores to the re-rank threads)
  RBQ_HIP(hipEventCreateWithFlags(&got->done, hipEventDisableTiming | hipEventBlockingSync));
  return got;
}

void ws_release(rbq_index* idx, std::unique_ptr<Workspace> ws, hipStream_t s) {
  if (!ws) return;
  RBQ_HIP(hipEventRecord(ws->done, s));
  std::lock_guard<std::mutex> g(idx->ws_mu);
  idx->ws_free.push_back(std::move(ws));
}

// Copies n rows of d floats (host or device source, rows packed) into a
// device array with row stride ld. Host sources go through 1-D copies (one per
// chunk of rows) because a pitched copy from pageable memory moves one row at
// a time.
void upload_rows(float* dst, int ld, const float* src, int d, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const bool dev = is_device_ptr(src);
  if (ld == d) {
    RBQ_HIP(hipMemcpyAsync(dst, src, (size_t)n * d * sizeof(float),
                           dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    return;
  }
  if (dev) {
    RBQ_HIP(hipMemcpy2DAsync(dst, ld * sizeof(float), src, d * sizeof(float), d * sizeof(float), n,
                             hipMemcpyDeviceToDevice, s));
    return;
  }
  const int64_t chunk = std::min<int64_t>(n, 1 << 18);
  DevBuf tmp;
  tmp.alloc((size_t)chunk * d * sizeof(float));
  for (int64_t r = 0; r < n; r += chunk) {
    const int64_t m = std::min(chunk, n - r);
    RBQ_HIP(hipMemcpyAsync(tmp.p, src + (size_t)r * d, (size_t)m * d * sizeof(float),
                           hipMemcpyHostToDevice, s));
    RBQ_HIP(hipMemcpy2DAsync(dst + (size_t)r * ld, ld * sizeof(float), tmp.p, d * sizeof(float),
                             d * sizeof(float), m, hipMemcpyDeviceToDevice, s));
    RBQ_HIP(hipStreamSynchronize(s));  // tmp is reused by the next chunk
  }
}

namespace {

struct StreamGuard {
  hipStream_t s = nullptr;
  StreamGuard() { RBQ_HIP(hipStreamCreate(&s)); }
  ~StreamGuard() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

__global__ void k_count_nonfinite(const float* X, int64_t rows, int d, int ld, unsigned* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = rows * d;
  unsigned bad = 0;
  for (int64_t e = t; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d;
    const float v = X[r * ld + (e - r * d)];
    bad += !isfinite(v);
  }
  if (bad) atomicAdd(out, bad);
}

// Device k-means (Sec. 3.1.1 Phases 1-2). Returns nlist x ld host centroids.
std::vector<float> kmeans_gpu(const float* Xd, int64_t n, int d, int ld, int nlist,
                              const rbq_build_params& p, Rng& rng, hipStream_t s) {
  const int64_t tn = p.train_n > 0 ? std::min<int64_t>(n, p.train_n)
                                   : std::min<int64_t>(n, (int64_t)256 * nlist);
  RBQ_CHECK(tn >= nlist, "k-means training sample is smaller than nlist");
  const int iters = p.kmeans_iters > 0 ? p.kmeans_iters : 25;
  const int restarts = p.kmeans_restarts > 0 ? p.kmeans_restarts : 3;
  const std::vector<int64_t> sample = sample_without_replacement(n, tn, rng);

  DevBuf didx, T, dC, dcn, keys, mind, bsum, pick;
  didx.alloc(tn * sizeof(int64_t));
  T.alloc((size_t)tn * ld * sizeof(float));
  RBQ_HIP(hipMemcpyAsync(didx.p, sample.data(), tn * sizeof(int64_t), hipMemcpyHostToDevice, s));
  launch_gather_rows(s, Xd, ld, didx.as<int64_t>(), tn, T.as<float>(), ld);
  std::vector<float> hT((size_t)tn * ld);
  RBQ_HIP(hipMemcpyAsync(hT.data(), T.p, hT.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  RBQ_HIP(hipStreamSynchronize(s));
  std::vector<double> tnorm(tn);
  for (int64_t t = 0; t < tn; ++t) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) acc += (double)hT[t * ld + k] * hT[t * ld + k];
    tnorm[t] = acc;
  }
  const int64_t nb = (tn + 255) / 256;
  dC.alloc((size_t)nlist * ld * sizeof(float));
  dcn.alloc(nlist * sizeof(float));
  keys.alloc(tn * sizeof(uint64_t));
  mind.alloc(tn * sizeof(float));
  bsum.alloc(nb * sizeof(double));
  pick.alloc(sizeof(int64_t));

  std::vector<float> hC((size_t)nlist * ld, 0.f), best;
  std::vector<float> hcn(nlist);
  std::vector<uint64_t> hk(tn);
  std::vector<int32_t> a(tn), prev;
  std::vector<double> dist(tn);
  double best_obj = INFINITY;

  auto assign_train = [&]() -> double {
    for (int j = 0; j < nlist; ++j) {
      double acc = 0.0;
      for (int k = 0; k < d; ++k) acc += (double)hC[(size_t)j * ld + k] * hC[(size_t)j * ld + k];
      hcn[j] = (float)acc;
    }
    RBQ_HIP(hipMemcpyAsync(dC.p, hC.data(), hC.size() * sizeof(float), hipMemcpyHostToDevice, s));
    RBQ_HIP(hipMemcpyAsync(dcn.p, hcn.data(), nlist * sizeof(float), hipMemcpyHostToDevice, s));
    launch_assign_argmin(s, T.as<float>(), ld, dC.as<float>(), ld, dcn.as<float>(), (int)tn, nlist,
                         ld, keys.as<uint64_t>());
    RBQ_HIP(hipMemcpyAsync(hk.data(), keys.p, tn * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    RBQ_HIP(hipStreamSynchronize(s));
    double obj = 0.0;
    for (int64_t t = 0; t < tn; ++t) {
      a[t] = (int32_t)(uint32_t)hk[t];
      dist[t] = std::max(0.0, (double)f32_ord((uint32_t)(hk[t] >> 32)) + tnorm[t]);
      obj += dist[t];
    }
    return obj;
  };

  // k-means++ seeding runs on an evenly strided subset of at most 32 nlist
  // training rows (the training rows are already a uniform random sample)
  const int64_t sn = p.kmeans_init == 1 ? tn : std::min<int64_t>(tn, (int64_t)32 * nlist);
  DevBuf S;
  const float* Sd = T.as<float>();
  if (sn < tn) {
    std::vector<int64_t> sub(sn);
    for (int64_t t = 0; t < sn; ++t) sub[t] = t * tn / sn;
    DevBuf dsub;
    dsub.alloc(sn * sizeof(int64_t));
    S.alloc((size_t)sn * ld * sizeof(float));
    RBQ_HIP(hipMemcpyAsync(dsub.p, sub.data(), sn * sizeof(int64_t), hipMemcpyHostToDevice, s));
    launch_gather_rows(s, T.as<float>(), ld, dsub.as<int64_t>(), sn, S.as<float>(), ld);
    RBQ_HIP(hipStreamSynchronize(s));
    Sd = S.as<float>();
  }
  for (int rs = 0; rs < restarts; ++rs) {
    if (p.kmeans_init == 1) {
      // random initial centroids (Sec. 3.1.1 Phase 1): nlist distinct
      // training rows, uniformly
      const std::vector<int64_t> rows = sample_without_replacement(tn, nlist, rng);
      for (int j = 0; j < nlist; ++j)
        std::memcpy(&hC[(size_t)j * ld], &hT[(size_t)rows[j] * ld], (size_t)ld * sizeof(float));
    } else {
      // k-means++ seeding on the device: first centre uniform, then D(x)^2 sampling
      RBQ_HIP(hipMemsetAsync(dC.p, 0, dC.bytes, s));
      const int64_t first = (int64_t)rng.below((uint64_t)sn);
      RBQ_HIP(hipMemcpyAsync(pick.p, &first, sizeof(int64_t), hipMemcpyHostToDevice, s));
      launch_copy_row(s, Sd, ld, pick.as<int64_t>(), dC.as<float>(), d);
      launch_kpp_update(s, Sd, ld, sn, d, pick.as<int64_t>(), mind.as<float>(), bsum.as<double>(), 1);
      for (int j = 1; j < nlist; ++j) {
        launch_kpp_choose(s, mind.as<float>(), bsum.as<double>(), sn, rng.uniform(), pick.as<int64_t>());
        launch_copy_row(s, Sd, ld, pick.as<int64_t>(), dC.as<float>() + (size_t)j * ld, d);
        launch_kpp_update(s, Sd, ld, sn, d, pick.as<int64_t>(), mind.as<float>(), bsum.as<double>(), 0);
      }
      RBQ_HIP(hipMemcpyAsync(hC.data(), dC.p, hC.size() * sizeof(float), hipMemcpyDeviceToHost, s));
      RBQ_HIP(hipStreamSynchronize(s));
    }
    build_log("k-means restart %d of %d: %lld training rows, %d lists, initial centroids set", rs + 1, restarts,
              (long long)tn, nlist);
    prev.clear();
    for (int it = 0; it < iters; ++it) {
      const double o = assign_train();
      build_log("k-means restart %d iteration %d of %d: objective %.6g", rs + 1, it + 1, iters, o);
      if (!prev.empty() && prev == a) break;
      lloyd_update(hT.data(), tn, d, ld, a.data(), dist.data(), nlist, hC.data());
      prev = a;
    }
    const double obj = assign_train();
    if (obj < best_obj) {
      best_obj = obj;
      best = hC;
    }
  }
  return best;
}

}  // namespace

rbq_index* build_index(const float* x, int64_t n, int d, const rbq_build_params& p) {
  auto idx = std::make_unique<rbq_index>();
  RBQ_HIP(hipGetDevice(&idx->device));
  RBQ_HIP(hipDeviceGetAttribute(&idx->num_cus, hipDeviceAttributeMultiprocessorCount, idx->device));
  {
    size_t free_b = 0, total_b = 0;
    RBQ_HIP(hipMemGetInfo(&free_b, &total_b));
    idx->device_mem = (int64_t)total_b;
  }
  idx->n = n;
  idx->d = d;
  idx->ld = (int)round_up(d, 4);
  idx->nlist = p.nlist;
  idx->bq = p.bq;
  idx->bqs = p.bq <= 4 ? 4 : 8;
  idx->W = (d + 31) / 32;
  idx->vectors_on_host = p.vectors_on_host;  // -1 (automatic) is settled once the index is built
  idx->host_threads = p.host_threads;
  const int ld = idx->ld, nlist = p.nlist, W = idx->W;
  StreamGuard sg;
  hipStream_t s = sg.s;
  Rng rng(p.seed);

  // raw vectors on the device, rows padded to ld with zeros (kept as the
  // index's own copy when they stay in HBM)
  DevBuf& Xd = idx->X;
  Xd.alloc((size_t)n * ld * sizeof(float));
  if (ld != d) RBQ_HIP(hipMemsetAsync(Xd.p, 0, Xd.bytes, s));
  upload_rows(Xd.as<float>(), ld, x, d, n, s);
  build_log("%lld x %d rows staged on the device", (long long)n, d);
  {
    DevBuf bad;
    bad.alloc(sizeof(unsigned));
    RBQ_HIP(hipMemsetAsync(bad.p, 0, sizeof(unsigned), s));
    hipLaunchKernelGGL(k_count_nonfinite, dim3(1024), dim3(256), 0, s, Xd.as<float>(), n, d, ld,
                       bad.as<unsigned>());
    RBQ_HIP(hipGetLastError());
    unsigned hb = 0;
    RBQ_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
    RBQ_HIP(hipStreamSynchronize(s));
    RBQ_CHECK(hb == 0, "input vectors contain NaN or Inf");
  }

  // centroids
  std::vector<float> hCld((size_t)nlist * ld, 0.f);
  if (p.centroids) {
    for (int j = 0; j < nlist; ++j)
      for (int k = 0; k < d; ++k) {
        const float v = p.centroids[(size_t)j * d + k];
        RBQ_CHECK(std::isfinite(v), "centroids contain NaN or Inf");
        hCld[(size_t)j * ld + k] = v;
      }
  } else {
    hCld = kmeans_gpu(Xd.as<float>(), n, d, ld, nlist, p, rng, s);
  }
  idx->hC.resize((size_t)nlist * d);
  for (int j = 0; j < nlist; ++j)
    for (int k = 0; k < d; ++k) idx->hC[(size_t)j * d + k] = hCld[(size_t)j * ld + k];
  idx->C.alloc(hCld.size() * sizeof(float));
  RBQ_HIP(hipMemcpyAsync(idx->C.p, hCld.data(), hCld.size() * sizeof(float), hipMemcpyHostToDevice, s));

  // rotation P (row-major), stored transposed: Pt[i][k] = P[k][i]
  idx->hP.resize((size_t)d * d);
  if (p.rotation) {
    for (size_t t = 0; t < idx->hP.size(); ++t) {
      RBQ_CHECK(std::isfinite(p.rotation[t]), "rotation contains NaN or Inf");
      idx->hP[t] = p.rotation[t];
    }
  } else {
    Rng prng(p.seed ^ 0x5D1E5EEDull);
    const std::vector<double> P64 = haar_orthogonal(d, prng);
    for (size_t t = 0; t < P64.size(); ++t) idx->hP[t] = (float)P64[t];
  }
  std::vector<float> hPt((size_t)d * ld, 0.f);
  for (int k = 0; k < d; ++k)
    for (int i = 0; i < d; ++i) hPt[(size_t)i * ld + k] = idx->hP[(size_t)k * d + i];
  idx->Pt.alloc(hPt.size() * sizeof(float));
  RBQ_HIP(hipMemcpyAsync(idx->Pt.p, hPt.data(), hPt.size() * sizeof(float), hipMemcpyHostToDevice, s));

  // rotated centroids and squared norms (FP64 sums, stored FP32)
  idx->Crot.alloc((size_t)nlist * ld * sizeof(float));
  idx->cnorm.alloc(nlist * sizeof(float));
  RBQ_HIP(hipMemsetAsync(idx->Crot.p, 0, idx->Crot.bytes, s));
  launch_rotate_rows_f64(s, idx->C.as<float>(), ld, idx->Pt.as<float>(), ld, nlist, d,
                         idx->Crot.as<float>(), ld, idx->cnorm.as<float>());

  // assignment: given, or nearest centroid on the GPU
  idx->h_assign.resize(n);
  if (p.assignment) {
    for (int64_t i = 0; i < n; ++i) {
      RBQ_CHECK(p.assignment[i] >= 0 && p.assignment[i] < nlist, "assignment out of range");
      idx->h_assign[i] = p.assignment[i];
    }
  } else {
    DevBuf keys;
    keys.alloc(n * sizeof(uint64_t));
    // in launches of 16M rows (each a few seconds at the largest list counts)
    const int64_t step = int64_t(1) << 24;
    for (int64_t r0 = 0; r0 < n; r0 += step) {
      const int64_t m = std::min(step, n - r0);
      launch_assign_argmin(s, Xd.as<float>() + (size_t)r0 * ld, ld, idx->C.as<float>(), ld,
                           idx->cnorm.as<float>(), (int)m, nlist, ld, keys.as<uint64_t>() + r0);
      if (build_log_on()) {
        RBQ_HIP(hipStreamSynchronize(s));
        build_log("assignment: %lld of %lld rows", (long long)(r0 + m), (long long)n);
      }
    }
    std::vector<uint64_t> hk(n);
    RBQ_HIP(hipMemcpyAsync(hk.data(), keys.p, n * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
    RBQ_HIP(hipStreamSynchronize(s));
    for (int64_t i = 0; i < n; ++i) idx->h_assign[i] = (int32_t)(uint32_t)hk[i];
  }

  // lists: stable counting sort by list id (ids ascend inside each list), each
  // list padded to whole 64-vector micro-blocks
  std::vector<int64_t> cnt(nlist, 0);
  for (int64_t i = 0; i < n; ++i) ++cnt[idx->h_assign[i]];
  idx->h_list_len.resize(nlist);
  idx->h_list_mb.resize(nlist);
  int64_t nmb = 0;
  for (int j = 0; j < nlist; ++j) {
    idx->h_list_len[j] = (int32_t)cnt[j];
    idx->h_list_mb[j] = (int32_t)nmb;
    nmb += ceil_div(cnt[j], MB);
    idx->max_list_len = std::max<int64_t>(idx->max_list_len, cnt[j]);
  }
  RBQ_CHECK(nmb * MB < (int64_t)INT32_MAX, "index too large for 32-bit positions");
  idx->nmb = nmb;
  idx->h_pos2id.assign(nmb * MB, -1);
  std::vector<int32_t> mb_list(nmb);
  {
    std::vector<int64_t> fill(nlist);
    for (int j = 0; j < nlist; ++j) {
      fill[j] = (int64_t)idx->h_list_mb[j] * MB;
      for (int64_t m = idx->h_list_mb[j]; m < idx->h_list_mb[j] + ceil_div(cnt[j], MB); ++m) mb_list[m] = j;
    }
    for (int64_t i = 0; i < n; ++i) idx->h_pos2id[fill[idx->h_assign[i]]++] = (int32_t)i;
  }
  idx->list_len.alloc(nlist * sizeof(int32_t));
  idx->list_mb.alloc(nlist * sizeof(int32_t));
  idx->pos2id.alloc(idx->h_pos2id.size() * sizeof(int32_t));
  DevBuf dmb;
  dmb.alloc(std::max<int64_t>(1, nmb) * sizeof(int32_t));
  RBQ_HIP(hipMemcpyAsync(idx->list_len.p, idx->h_list_len.data(), nlist * sizeof(int32_t), hipMemcpyHostToDevice, s));
  RBQ_HIP(hipMemcpyAsync(idx->list_mb.p, idx->h_list_mb.data(), nlist * sizeof(int32_t), hipMemcpyHostToDevice, s));
  RBQ_HIP(hipMemcpyAsync(idx->pos2id.p, idx->h_pos2id.data(), idx->h_pos2id.size() * sizeof(int32_t),
                         hipMemcpyHostToDevice, s));
  if (nmb) RBQ_HIP(hipMemcpyAsync(dmb.p, mb_list.data(), nmb * sizeof(int32_t), hipMemcpyHostToDevice, s));

  // RaBitQ encoding of every micro-block
  const size_t rec = (size_t)(W + 2) * MB;
  idx->blocks.alloc(std::max<int64_t>(1, nmb) * rec * sizeof(uint32_t));
  idx->nx.alloc(std::max<int64_t>(1, nmb) * MB * sizeof(float));
  idx->alpha.alloc(std::max<int64_t>(1, nmb) * MB * sizeof(float));
  const int64_t step = 1 << 20;
  for (int64_t m0 = 0; m0 < nmb; m0 += step)
    launch_encode(s, Xd.as<float>(), ld, idx->C.as<float>(), ld, idx->Pt.as<float>(), ld,
                  idx->pos2id.as<int32_t>(), dmb.as<int32_t>(), m0, std::min(nmb, m0 + step), d, W,
                  idx->blocks.as<uint32_t>(), idx->nx.as<float>(), idx->alpha.as<float>());

  if (build_log_on()) {
    RBQ_HIP(hipStreamSynchronize(s));
    build_log("encoded %lld micro-blocks", (long long)nmb);
  }
  if (p.ivf_flat) {  // the lists' full-precision rows, for the IVF-Flat scan
    idx->flat.alloc(std::max<int64_t>(1, nmb) * (int64_t)(flat_dp(d) + 1) * MB * sizeof(float));
    launch_flat_fill(s, Xd.as<float>(), ld, idx->pos2id.as<int32_t>(), nmb, d, idx->flat.as<float>());
  }
  RBQ_HIP(hipStreamSynchronize(s));
  if (idx->vectors_on_host < 0) {
    // automatic placement: HBM if the raw vectors (already resident) leave
    // enough device memory free for search workspaces, else the host
    size_t free_b = 0, total_b = 0;
    RBQ_HIP(hipMemGetInfo(&free_b, &total_b));
    const size_t reserve = std::max<size_t>((size_t)8 << 30, total_b / 8);
    idx->vectors_on_host = free_b >= reserve ? 0 : 1;
  }
  if (idx->vectors_on_host) {
    if (p.borrow_vectors) {
      idx->hostX = const_cast<float*>(x);  // the caller's host rows
      idx->hostX_owned = false;
    } else {
      const size_t count = (size_t)n * d;
      idx->hostX = host_rows_alloc(count * sizeof(float), &idx->hostX_mapped);
      if (!is_device_ptr(x)) {
        const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
        host_rows_fill(idx->hostX, x, count, std::min(hw, 16));
      } else if (ld == d) {
        RBQ_HIP(hipMemcpyAsync(idx->hostX, Xd.p, count * sizeof(float), hipMemcpyDeviceToHost, s));
      } else {
        RBQ_HIP(hipMemcpy2DAsync(idx->hostX, d * sizeof(float), Xd.p, ld * sizeof(float),
                                 d * sizeof(float), n, hipMemcpyDeviceToHost, s));
      }
      RBQ_HIP(hipStreamSynchronize(s));
    }
    Xd.reset();
  }
  compact_raw_vectors(idx.get(), s);
  return idx.release();
}

void compact_raw_vectors(rbq_index* idx, hipStream_t s) {
  if (idx->vectors_on_host || !idx->X.p) return;
  DevBuf bad;
  bad.alloc(sizeof(unsigned));
  RBQ_HIP(hipMemsetAsync(bad.p, 0, sizeof(unsigned), s));
  launch_count_not_u8(s, idx->X.as<float>(), idx->n, idx->d, idx->ld, bad.as<unsigned>());
  unsigned hb = 0;
  RBQ_HIP(hipMemcpyAsync(&hb, bad.p, sizeof(unsigned), hipMemcpyDeviceToHost, s));
  RBQ_HIP(hipStreamSynchronize(s));
  if (hb != 0) return;
  idx->X8.alloc((size_t)idx->n * idx->ld);
  launch_to_u8(s, idx->X.as<float>(), (int64_t)idx->n * idx->ld, idx->X8.as<uint8_t>());
  RBQ_HIP(hipStreamSynchronize(s));
  idx->X.reset();
}

}  // namespace rbq

rbq_index::~rbq_index() {
  pool.reset();
  if (host_gpu_stream) (void)hipStreamDestroy(host_gpu_stream);
  if (host_copy_stream) (void)hipStreamDestroy(host_copy_stream);
  for (auto& pf : pinned_free) (void)hipHostFree(pf.first);
  if (hostX && hostX_owned) rbq::host_rows_free(hostX, hostX_mapped);
}
