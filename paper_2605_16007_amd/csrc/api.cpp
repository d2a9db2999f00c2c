// The C ABI of librbq: argument validation, status codes and thread-local
// error messages around the C++ implementation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>

#include "index.hpp"
#include "server.hpp"

namespace {

thread_local std::string g_err;

template <class F>
rbq_status guarded(F&& f) {
  g_err.clear();
  try {
    f();
    return RBQ_OK;
  } catch (const rbq::Error& e) {
    g_err = e.what();
    // (a failed runtime call, such as an allocation that did not fit, also
    // stays as the thread's last HIP error: clear it so that the next call's
    // launch checks do not report it again)
    (void)hipGetLastError();
    return e.status;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return RBQ_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    (void)hipGetLastError();
    return RBQ_EDEVICE;
  }
}

rbq_status invalid(const char* msg) {
  g_err = msg;
  return RBQ_EINVAL;
}

void check_search_args(const rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                       int32_t rerank_n) {
  RBQ_CHECK(idx != nullptr, "index is NULL");
  RBQ_CHECK(nq >= 0, "nq must be >= 0");
  RBQ_CHECK(nq == 0 || q != nullptr, "queries are NULL");
  RBQ_CHECK(nprobe >= 1 && nprobe <= idx->nlist, "nprobe must be in [1, nlist]");
  RBQ_CHECK(nprobe <= rbq::MAX_SEL, "nprobe must be <= 4096");
  RBQ_CHECK(rerank_n >= 1 && rerank_n <= rbq::MAX_R, "rerank_n must be in [1, 3840]");
  RBQ_CHECK(k >= 1 && k <= rerank_n, "k must be in [1, rerank_n]");
  RBQ_CHECK(nq * (int64_t)nprobe <= (int64_t)INT32_MAX, "nq * nprobe too large");
}

uint64_t fnv1a(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

namespace rbq {

void export_item(const rbq_index* idx, int what, void* dst, size_t bytes) {
  RBQ_CHECK(dst != nullptr, "export destination is NULL");
  const int64_t n = idx->n;
  const int d = idx->d, W = idx->W;
  RBQ_HIP(hipSetDevice(idx->device));
  auto need = [&](size_t b) { RBQ_CHECK(bytes == b, "export size mismatch"); };
  switch (what) {
    case RBQ_EXPORT_CENTROIDS:
      need(idx->hC.size() * sizeof(float));
      std::memcpy(dst, idx->hC.data(), bytes);
      break;
    case RBQ_EXPORT_ROTATION:
      need(idx->hP.size() * sizeof(float));
      std::memcpy(dst, idx->hP.data(), bytes);
      break;
    case RBQ_EXPORT_ASSIGN:
      need(n * sizeof(int32_t));
      std::memcpy(dst, idx->h_assign.data(), bytes);
      break;
    case RBQ_EXPORT_LIST_SIZES: {
      need(idx->nlist * sizeof(int64_t));
      int64_t* o = static_cast<int64_t*>(dst);
      for (int j = 0; j < idx->nlist; ++j) o[j] = idx->h_list_len[j];
      break;
    }
    case RBQ_EXPORT_CODES: {
      const int cb = (d + 7) / 8;
      need((size_t)n * cb);
      const size_t rec = (size_t)(W + 2) * MB;
      std::vector<uint32_t> blk(idx->nmb * rec);
      RBQ_HIP(hipMemcpy(blk.data(), idx->blocks.p, blk.size() * sizeof(uint32_t), hipMemcpyDeviceToHost));
      uint8_t* o = static_cast<uint8_t*>(dst);
      for (int64_t pos = 0; pos < idx->nmb * MB; ++pos) {
        const int id = idx->h_pos2id[pos];
        if (id < 0) continue;
        const int64_t m = pos / MB, lane = pos % MB;
        for (int byte = 0; byte < cb; ++byte) {
          const uint32_t w = blk[m * rec + (size_t)(byte >> 2) * MB + lane];
          o[(size_t)id * cb + byte] = (uint8_t)(w >> (8 * (byte & 3)));
        }
      }
      break;
    }
    case RBQ_EXPORT_FACTORS: {
      need((size_t)n * 2 * sizeof(float));
      std::vector<float> nx(idx->nmb * MB), al(idx->nmb * MB);
      RBQ_HIP(hipMemcpy(nx.data(), idx->nx.p, nx.size() * sizeof(float), hipMemcpyDeviceToHost));
      RBQ_HIP(hipMemcpy(al.data(), idx->alpha.p, al.size() * sizeof(float), hipMemcpyDeviceToHost));
      float* o = static_cast<float*>(dst);
      for (int64_t pos = 0; pos < idx->nmb * MB; ++pos) {
        const int id = idx->h_pos2id[pos];
        if (id < 0) continue;
        o[(size_t)id * 2] = nx[pos];
        o[(size_t)id * 2 + 1] = al[pos];
      }
      break;
    }
    default:
      fail(RBQ_EINVAL, "unknown export item");
  }
}

// ---- persistence: magic, header, then tagged sections with FNV-1a checksums.

namespace {
constexpr char MAGIC[8] = {'R', 'B', 'Q', 'I', 'D', 'X', '0', '1'};
struct Header {
  int64_t n, nmb, max_list_len;
  int32_t d, nlist, bq, vectors_on_host;
};

void put_section(std::ofstream& f, uint32_t tag, const void* p, uint64_t bytes) {
  const uint64_t h = fnv1a(p, bytes);
  f.write(reinterpret_cast<const char*>(&tag), 4);
  f.write(reinterpret_cast<const char*>(&bytes), 8);
  f.write(reinterpret_cast<const char*>(&h), 8);
  f.write(static_cast<const char*>(p), (std::streamsize)bytes);
}

void get_section(std::ifstream& f, uint32_t tag, void* p, uint64_t bytes) {
  uint32_t t = 0;
  uint64_t b = 0, h = 0;
  f.read(reinterpret_cast<char*>(&t), 4);
  f.read(reinterpret_cast<char*>(&b), 8);
  f.read(reinterpret_cast<char*>(&h), 8);
  RBQ_CHECK(f && t == tag && b == bytes, "index file: unexpected section");
  f.read(static_cast<char*>(p), (std::streamsize)bytes);
  RBQ_CHECK((bool)f, "index file truncated");
  RBQ_CHECK(fnv1a(p, bytes) == h, "index file: checksum mismatch");
}
}  // namespace

void save_index(const rbq_index* idx, const char* path) {
  RBQ_HIP(hipSetDevice(idx->device));
  std::ofstream f(path, std::ios::binary);
  RBQ_CHECK((bool)f, "cannot open index file for writing");
  f.write(MAGIC, 8);
  const Header h{idx->n, idx->nmb, idx->max_list_len, idx->d, idx->nlist, idx->bq, idx->vectors_on_host};
  f.write(reinterpret_cast<const char*>(&h), sizeof(h));
  const size_t rec = (size_t)(idx->W + 2) * MB;
  std::vector<uint32_t> blk(idx->nmb * rec);
  RBQ_HIP(hipMemcpy(blk.data(), idx->blocks.p, blk.size() * 4, hipMemcpyDeviceToHost));
  std::vector<float> nx(idx->nmb * MB), al(idx->nmb * MB), X((size_t)idx->n * idx->d);
  RBQ_HIP(hipMemcpy(nx.data(), idx->nx.p, nx.size() * 4, hipMemcpyDeviceToHost));
  RBQ_HIP(hipMemcpy(al.data(), idx->alpha.p, al.size() * 4, hipMemcpyDeviceToHost));
  if (idx->vectors_on_host) {
    std::memcpy(X.data(), idx->hostX, X.size() * 4);
  } else if (idx->X8.p) {  // byte form: the values are the integers themselves
    std::vector<uint8_t> x8((size_t)idx->n * idx->d);
    RBQ_HIP(hipMemcpy2D(x8.data(), idx->d, idx->X8.p, idx->ld, idx->d, idx->n, hipMemcpyDeviceToHost));
    for (size_t e = 0; e < X.size(); ++e) X[e] = (float)x8[e];
  } else {
    RBQ_HIP(hipMemcpy2D(X.data(), idx->d * 4, idx->X.p, idx->ld * 4, idx->d * 4, idx->n, hipMemcpyDeviceToHost));
  }
  put_section(f, 1, idx->hC.data(), idx->hC.size() * 4);
  put_section(f, 2, idx->hP.data(), idx->hP.size() * 4);
  put_section(f, 3, idx->h_assign.data(), idx->h_assign.size() * 4);
  put_section(f, 4, idx->h_list_len.data(), idx->h_list_len.size() * 4);
  put_section(f, 5, idx->h_list_mb.data(), idx->h_list_mb.size() * 4);
  put_section(f, 6, idx->h_pos2id.data(), idx->h_pos2id.size() * 4);
  put_section(f, 7, blk.data(), blk.size() * 4);
  put_section(f, 8, nx.data(), nx.size() * 4);
  put_section(f, 9, al.data(), al.size() * 4);
  put_section(f, 10, X.data(), X.size() * 4);
  RBQ_CHECK((bool)f, "write failed");
}

rbq_index* load_index(const char* path) {
  std::ifstream f(path, std::ios::binary);
  RBQ_CHECK((bool)f, "cannot open index file");
  char magic[8];
  f.read(magic, 8);
  RBQ_CHECK(f && std::memcmp(magic, MAGIC, 8) == 0, "not an rbq index file (or another version)");
  Header h;
  f.read(reinterpret_cast<char*>(&h), sizeof(h));
  RBQ_CHECK(f && h.n > 0 && h.d > 0 && h.nlist > 0 && h.bq >= 1 && h.bq <= 8, "bad index header");
  auto idx = std::make_unique<rbq_index>();
  RBQ_HIP(hipGetDevice(&idx->device));
  RBQ_HIP(hipDeviceGetAttribute(&idx->num_cus, hipDeviceAttributeMultiprocessorCount, idx->device));
  {
    size_t free_b = 0, total_b = 0;
    RBQ_HIP(hipMemGetInfo(&free_b, &total_b));
    idx->device_mem = (int64_t)total_b;
  }
  idx->n = h.n;
  idx->d = h.d;
  idx->ld = (int)round_up(h.d, 4);
  idx->nlist = h.nlist;
  idx->bq = h.bq;
  idx->bqs = h.bq <= 4 ? 4 : 8;
  idx->W = (h.d + 31) / 32;
  idx->nmb = h.nmb;
  idx->max_list_len = h.max_list_len;
  idx->vectors_on_host = h.vectors_on_host;
  const int d = idx->d, ld = idx->ld, nlist = idx->nlist;
  idx->hC.resize((size_t)nlist * d);
  idx->hP.resize((size_t)d * d);
  idx->h_assign.resize(h.n);
  idx->h_list_len.resize(nlist);
  idx->h_list_mb.resize(nlist);
  idx->h_pos2id.resize(h.nmb * MB);
  const size_t rec = (size_t)(idx->W + 2) * MB;
  std::vector<uint32_t> blk(h.nmb * rec);
  std::vector<float> nx(h.nmb * MB), al(h.nmb * MB), X((size_t)h.n * d);
  get_section(f, 1, idx->hC.data(), idx->hC.size() * 4);
  get_section(f, 2, idx->hP.data(), idx->hP.size() * 4);
  get_section(f, 3, idx->h_assign.data(), idx->h_assign.size() * 4);
  get_section(f, 4, idx->h_list_len.data(), idx->h_list_len.size() * 4);
  get_section(f, 5, idx->h_list_mb.data(), idx->h_list_mb.size() * 4);
  get_section(f, 6, idx->h_pos2id.data(), idx->h_pos2id.size() * 4);
  get_section(f, 7, blk.data(), blk.size() * 4);
  get_section(f, 8, nx.data(), nx.size() * 4);
  get_section(f, 9, al.data(), al.size() * 4);
  get_section(f, 10, X.data(), X.size() * 4);
  // device copies
  std::vector<float> Cld((size_t)nlist * ld, 0.f), Pt((size_t)d * ld, 0.f);
  for (int j = 0; j < nlist; ++j)
    for (int t = 0; t < d; ++t) Cld[(size_t)j * ld + t] = idx->hC[(size_t)j * d + t];
  for (int r = 0; r < d; ++r)
    for (int i = 0; i < d; ++i) Pt[(size_t)i * ld + r] = idx->hP[(size_t)r * d + i];
  idx->C.alloc(Cld.size() * 4);
  idx->Pt.alloc(Pt.size() * 4);
  idx->Crot.alloc(Cld.size() * 4);
  idx->cnorm.alloc(nlist * 4);
  idx->list_len.alloc(nlist * 4);
  idx->list_mb.alloc(nlist * 4);
  idx->pos2id.alloc(idx->h_pos2id.size() * 4);
  idx->blocks.alloc(blk.size() * 4);
  idx->nx.alloc(nx.size() * 4);
  idx->alpha.alloc(al.size() * 4);
  RBQ_HIP(hipMemcpy(idx->C.p, Cld.data(), Cld.size() * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->Pt.p, Pt.data(), Pt.size() * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemset(idx->Crot.p, 0, idx->Crot.bytes));
  RBQ_HIP(hipMemcpy(idx->list_len.p, idx->h_list_len.data(), nlist * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->list_mb.p, idx->h_list_mb.data(), nlist * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->pos2id.p, idx->h_pos2id.data(), idx->h_pos2id.size() * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->blocks.p, blk.data(), blk.size() * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->nx.p, nx.data(), nx.size() * 4, hipMemcpyHostToDevice));
  RBQ_HIP(hipMemcpy(idx->alpha.p, al.data(), al.size() * 4, hipMemcpyHostToDevice));
  launch_rotate_rows_f64(nullptr, idx->C.as<float>(), ld, idx->Pt.as<float>(), ld, nlist, d,
                         idx->Crot.as<float>(), ld, idx->cnorm.as<float>());
  if (idx->vectors_on_host) {
    idx->hostX = host_rows_alloc(X.size() * 4, &idx->hostX_mapped);
    host_rows_fill(idx->hostX, X.data(), X.size(), 8);
  } else {
    idx->X.alloc((size_t)h.n * ld * 4);
    if (ld != d) RBQ_HIP(hipMemset(idx->X.p, 0, idx->X.bytes));
    RBQ_HIP(hipMemcpy2D(idx->X.p, ld * 4, X.data(), d * 4, d * 4, h.n, hipMemcpyHostToDevice));
  }
  RBQ_HIP(hipDeviceSynchronize());
  compact_raw_vectors(idx.get(), nullptr);
  return idx.release();
}

}  // namespace rbq

extern "C" {

void rbq_build_params_init(rbq_build_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->bq = 4;
  p->kmeans_iters = 25;
  p->kmeans_restarts = 3;
  p->vectors_on_host = -1;
}

rbq_status rbq_build_index(const float* x, int64_t n, int32_t d, const rbq_build_params* p,
                           rbq_index** out) {
  if (!out) return invalid("out is NULL");
  if (!x) return invalid("x is NULL");
  if (!p) return invalid("params are NULL");
  if (n < 1) return invalid("n must be >= 1");
  if (d < 1 || d > 4096) return invalid("d must be in [1, 4096]");
  if (p->nlist < 1 || p->nlist > n) return invalid("nlist must be in [1, n]");
  if (p->bq < 1 || p->bq > 8) return invalid("bq must be in [1, 8]");
  if (p->kmeans_iters < 0 || p->kmeans_restarts < 0 || p->train_n < 0)
    return invalid("k-means parameters must be >= 0");
  if (p->vectors_on_host < -1 || p->vectors_on_host > 1) return invalid("vectors_on_host must be -1, 0 or 1");
  if (p->borrow_vectors != 0 && p->borrow_vectors != 1) return invalid("borrow_vectors must be 0 or 1");
  if (p->ivf_flat != 0 && p->ivf_flat != 1) return invalid("ivf_flat must be 0 or 1");
  if (p->kmeans_init != 0 && p->kmeans_init != 1) return invalid("kmeans_init must be 0 or 1");
  if (p->ivf_flat && d > 256) return invalid("ivf_flat supports d <= 256");
  if (p->borrow_vectors) {
    if (p->vectors_on_host == 0) return invalid("borrow_vectors needs the vectors on the host (vectors_on_host 1 or -1)");
    if (rbq::is_device_ptr(x)) return invalid("borrow_vectors needs x in host memory, not device memory");
  }
  for (int r : p->reserved)
    if (r != 0) return invalid("reserved fields must be zero");
  if (n > (int64_t)INT32_MAX) return invalid("n must fit in 31 bits");
  *out = nullptr;
  return guarded([&] { *out = rbq::build_index(x, n, d, *p); });
}

rbq_status rbq_free_index(rbq_index* idx) {
  if (!idx) return invalid("index is NULL");
  return guarded([&] {
    (void)hipSetDevice(idx->device);
    (void)hipDeviceSynchronize();
    for (auto& a : idx->pending) {
      for (auto e : a.e) (void)hipEventDestroy(e);
      for (auto e : a.scan) (void)hipEventDestroy(e);
    }
    delete idx;
  });
}

rbq_status rbq_get_info(const rbq_index* idx, rbq_index_info* info) {
  if (!idx || !info) return invalid("NULL argument");
  info->n = idx->n;
  info->d = idx->d;
  info->nlist = idx->nlist;
  info->bq = idx->bq;
  info->vectors_on_host = idx->vectors_on_host;
  info->vectors_borrowed = idx->hostX && !idx->hostX_owned ? 1 : 0;
  info->reserved = 0;
  info->max_list_len = idx->max_list_len;
  info->code_bytes = (int64_t)idx->blocks.bytes;
  info->device_bytes = (int64_t)(idx->X.bytes + idx->X8.bytes + idx->C.bytes + idx->Crot.bytes + idx->cnorm.bytes +
                                 idx->Pt.bytes + idx->blocks.bytes + idx->list_mb.bytes +
                                 idx->list_len.bytes + idx->pos2id.bytes + idx->nx.bytes +
                                 idx->alpha.bytes + idx->flat.bytes);
  return RBQ_OK;
}

rbq_status rbq_search(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                      int32_t rerank_n, int64_t* ids, float* sqdist, void* stream) {
  return guarded([&] {
    check_search_args(idx, q, nq, nprobe, k, rerank_n);
    RBQ_CHECK(nq == 0 || (ids != nullptr && sqdist != nullptr), "outputs are NULL");
    rbq::search(idx, q, nq, nprobe, k, rerank_n, ids, sqdist, static_cast<hipStream_t>(stream),
                rbq::SearchIO{});
  });
}

rbq_status rbq_search_noalloc(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                              int32_t rerank_n, int64_t* ids, float* sqdist, void* stream) {
  return guarded([&] {
    check_search_args(idx, q, nq, nprobe, k, rerank_n);
    RBQ_CHECK(nq == 0 || (ids != nullptr && sqdist != nullptr), "outputs are NULL");
    rbq::search_noalloc(idx, q, nq, nprobe, k, rerank_n, ids, sqdist, static_cast<hipStream_t>(stream));
  });
}

rbq_status rbq_search_mixed(rbq_index* idx, const float* q, int64_t nq, const int32_t* nprobe,
                            const int32_t* k, const int32_t* rerank_n, int32_t k_stride,
                            int64_t* ids, float* sqdist, void* stream) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr, "index is NULL");
    RBQ_CHECK(nq >= 0, "nq must be >= 0");
    if (nq == 0) return;
    RBQ_CHECK(q && nprobe && k && rerank_n && ids && sqdist, "an argument is NULL");
    RBQ_CHECK(k_stride >= 1, "k_stride must be >= 1");
    int np = 0, R = 0;
    for (int64_t i = 0; i < nq; ++i) {
      RBQ_CHECK(nprobe[i] >= 1 && nprobe[i] <= std::min(idx->nlist, rbq::MAX_SEL),
                "nprobe[i] must be in [1, min(nlist, 4096)]");
      RBQ_CHECK(rerank_n[i] >= 1 && rerank_n[i] <= rbq::MAX_R, "rerank_n[i] must be in [1, 3840]");
      RBQ_CHECK(k[i] >= 1 && k[i] <= rerank_n[i] && k[i] <= k_stride,
                "k[i] must be in [1, min(rerank_n[i], k_stride)]");
      np = std::max(np, nprobe[i]);
      R = std::max(R, rerank_n[i]);
    }
    RBQ_CHECK(k_stride <= R, "k_stride must be <= the largest rerank_n");
    RBQ_CHECK(nq * (int64_t)np <= (int64_t)INT32_MAX, "nq * nprobe too large");
    rbq::SearchIO io;
    io.q_nprobe = nprobe;
    io.q_k = k;
    io.q_R = rerank_n;
    rbq::search(idx, q, nq, np, k_stride, R, ids, sqdist, static_cast<hipStream_t>(stream), io);
  });
}

rbq_status rbq_search_debug(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                            int32_t rerank_n, rbq_debug_io* io) {
  return guarded([&] {
    check_search_args(idx, q, nq, nprobe, k, rerank_n);
    RBQ_CHECK(io != nullptr, "debug io is NULL");
    RBQ_CHECK(!io->inject_qu || io->inject_scalars, "inject_qu needs inject_scalars");
    hipStream_t s = nullptr;
    RBQ_HIP(hipStreamCreate(&s));
    rbq::SearchIO sio;
    sio.dbg = io;
    try {
      rbq::search(idx, q, nq, nprobe, k, rerank_n, nullptr, nullptr, s, sio);
    } catch (...) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
      throw;
    }
    RBQ_HIP(hipStreamSynchronize(s));
    RBQ_HIP(hipStreamDestroy(s));
  });
}

rbq_status rbq_export(const rbq_index* idx, int32_t what, void* dst, size_t bytes) {
  if (!idx) return invalid("index is NULL");
  return guarded([&] { rbq::export_item(idx, what, dst, bytes); });
}

rbq_status rbq_set_timing(rbq_index* idx, int32_t enabled) {
  if (!idx) return invalid("index is NULL");
  return guarded([&] {
    RBQ_HIP(hipSetDevice(idx->device));
    std::lock_guard<std::mutex> g(idx->timing_mu);
    for (auto& a : idx->pending) {
      for (auto e : a.e) (void)hipEventDestroy(e);
      for (auto e : a.scan) (void)hipEventDestroy(e);
    }
    idx->pending.clear();
    idx->last = rbq_timings{};
    if (enabled) {
      if (!idx->tcounter.p) idx->tcounter.alloc(7 * sizeof(unsigned long long));
      RBQ_HIP(hipMemset(idx->tcounter.p, 0, 7 * sizeof(unsigned long long)));
    }
    idx->timing.store(enabled ? 1 : 0);
  });
}

rbq_status rbq_get_timings(rbq_index* idx, rbq_timings* t) {
  if (!idx || !t) return invalid("NULL argument");
  return guarded([&] {
    RBQ_HIP(hipSetDevice(idx->device));
    std::lock_guard<std::mutex> g(idx->timing_mu);
    for (auto& a : idx->pending) {
      RBQ_HIP(hipEventSynchronize(a.e[5]));
      float ms[5], tot = 0.f, scan = 0.f, gscan = 0.f, fscan = 0.f;
      for (int i = 0; i < 5; ++i) RBQ_HIP(hipEventElapsedTime(&ms[i], a.e[i], a.e[i + 1]));
      RBQ_HIP(hipEventElapsedTime(&tot, a.e[0], a.e[5]));
      for (size_t c = 0; c + 1 < a.scan.size(); c += 2) {
        float t = 0.f;
        RBQ_HIP(hipEventElapsedTime(&t, a.scan[c], a.scan[c + 1]));
        scan += t;
        if (a.scan_lm[c / 2] == 1) gscan += t;
        if (a.scan_lm[c / 2] == 2) fscan += t;
      }
      idx->last.group_scan_ms += gscan;
      idx->last.fused_scan_ms += fscan;
      idx->last.fused_launches += a.fused;
      idx->last.probe_ms += ms[0];
      idx->last.rotate_ms += ms[1];
      idx->last.quant_ms += ms[2];
      idx->last.scan_ms += scan;
      idx->last.merge_ms += ms[3] - scan;
      idx->last.rerank_ms += ms[4];
      idx->last.total_ms += tot;
      idx->last.searches += a.first_part ? 1 : 0;  // sub-batches of one search add up
      idx->last.group_launches += a.group;
      idx->last.popc_launches += a.popc;
      for (auto e : a.e) (void)hipEventDestroy(e);
      for (auto e : a.scan) (void)hipEventDestroy(e);
    }
    idx->pending.clear();
    if (idx->tcounter.p) {
      unsigned long long c[7] = {0, 0, 0, 0, 0, 0, 0};
      RBQ_HIP(hipDeviceSynchronize());
      RBQ_HIP(hipMemcpy(c, idx->tcounter.p, sizeof(c), hipMemcpyDeviceToHost));
      idx->last.scanned_vectors = (int64_t)c[0];
      idx->last.scan_bytes = (int64_t)c[0] * (idx->W * 4 + 8);
      idx->last.read_bytes = (int64_t)c[1];
      idx->last.group_vectors = (int64_t)c[2];
      idx->last.group_read_bytes = (int64_t)c[3];
      idx->last.fused_vectors = (int64_t)c[4];
      idx->last.fused_read_bytes = (int64_t)c[5];
      idx->last.redo_queries = (int64_t)c[6];
    }
    *t = idx->last;
  });
}

rbq_status rbq_set_option(rbq_index* idx, int32_t option, int64_t value) {
  if (!idx) return invalid("index is NULL");
  switch (option) {
    case RBQ_OPT_SCAN:
      if (value < 0 || value > 3) return invalid("RBQ_OPT_SCAN must be 0, 1, 2 or 3");
      idx->opt_scan.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_GROUP_MIN:
      if (value < 1 || value > (1 << 20)) return invalid("RBQ_OPT_GROUP_MIN must be in [1, 2^20]");
      idx->opt_group_min.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_POOL_CAP:
      if (value < 0) return invalid("RBQ_OPT_POOL_CAP must be >= 0");
      idx->opt_pool_cap.store(value);
      return RBQ_OK;
    case RBQ_OPT_ROTATION:
      if (value < 0 || value > 1) return invalid("RBQ_OPT_ROTATION must be 0 or 1");
      idx->opt_rotation.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_ESTIMATOR:
      if (value < 0 || value > 2) return invalid("RBQ_OPT_ESTIMATOR must be 0, 1 or 2");
      if (value == 1 && idx->d > rbq::scan_lut_max_d())
        return invalid("RBQ_OPT_ESTIMATOR 1 supports d <= 1024");
      if (value == 2 && !idx->flat.p) return invalid("RBQ_OPT_ESTIMATOR 2 needs an index built with ivf_flat");
      idx->opt_estimator.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_BLOCK:
      if (value < -1 || value > (1 << 20)) return invalid("RBQ_OPT_BLOCK must be in [-1, 2^20]");
      idx->opt_block.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_HOST_PARTS:
      if (value < 0 || value > 64) return invalid("RBQ_OPT_HOST_PARTS must be in [0, 64]");
      idx->opt_host_parts.store((int)value);
      return RBQ_OK;
    case RBQ_OPT_GROUP_SIZE:
      if (value < 0 || value > 64) return invalid("RBQ_OPT_GROUP_SIZE must be in [0, 64]");
      idx->opt_group_size.store((int)value);
      return RBQ_OK;
    default:
      return invalid("unknown option");
  }
}

rbq_status rbq_save(const rbq_index* idx, const char* path) {
  if (!idx || !path) return invalid("NULL argument");
  return guarded([&] { rbq::save_index(idx, path); });
}

rbq_status rbq_load(const char* path, rbq_index** out) {
  if (!path || !out) return invalid("NULL argument");
  *out = nullptr;
  return guarded([&] { *out = rbq::load_index(path); });
}

rbq_status rbq_autotune(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                        int32_t rerank_n, rbq_tune_result* out) {
  return guarded([&] {
    check_search_args(idx, q, nq, nprobe, k, rerank_n);
    RBQ_CHECK(nq >= 1, "nq must be >= 1");
    rbq::autotune(idx, q, nq, nprobe, k, rerank_n, out);
  });
}

rbq_status rbq_tune_save(rbq_index* idx, const char* path) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr && path != nullptr, "an argument is NULL");
    rbq::tune_save(idx, path);
  });
}

rbq_status rbq_tune_load(rbq_index* idx, const char* path, int32_t* loaded) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr && path != nullptr, "an argument is NULL");
    const int n = rbq::tune_load(idx, path);
    if (loaded) *loaded = n;
  });
}

rbq_status rbq_tune_clear(rbq_index* idx) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr, "index is NULL");
    std::lock_guard<std::mutex> g(idx->tune_mu);
    idx->tune.clear();
  });
}

rbq_status rbq_server_params_init(rbq_server_params* p) {
  if (!p) return invalid("params is NULL");
  rbq::server_params_default(p);
  return RBQ_OK;
}

rbq_status rbq_server_create(rbq_index* idx, const rbq_server_params* p, rbq_server** out) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr && p != nullptr && out != nullptr, "an argument is NULL");
    *out = nullptr;
    *out = rbq::server_create(idx, *p);
  });
}

rbq_status rbq_submit(rbq_server* srv, const float* q, int32_t nprobe, int32_t k, int32_t rerank_n,
                      uint64_t* ticket) {
  rbq_status st = RBQ_OK;
  const rbq_status g = guarded([&] {
    RBQ_CHECK(srv != nullptr, "server is NULL");
    st = rbq::server_submit(srv, q, nprobe, k, rerank_n, ticket);
    if (st == RBQ_EAGAIN) g_err = "request queue is full";
  });
  return g != RBQ_OK ? g : st;
}

rbq_status rbq_poll(rbq_server* srv, uint64_t ticket, int64_t* ids, float* sqdist, int32_t* done,
                    int64_t* latency_ns) {
  return guarded([&] {
    RBQ_CHECK(srv != nullptr && done != nullptr, "server or done is NULL");
    RBQ_CHECK(ids != nullptr && sqdist != nullptr, "outputs are NULL");
    *done = 0;
    *done = rbq::server_collect(srv, ticket, ids, sqdist, 0, nullptr, latency_ns);
  });
}

rbq_status rbq_wait(rbq_server* srv, uint64_t ticket, int64_t* ids, float* sqdist,
                    int64_t timeout_us, int64_t* latency_ns) {
  int got = 0;
  const rbq_status g = guarded([&] {
    RBQ_CHECK(srv != nullptr, "server is NULL");
    RBQ_CHECK(ids != nullptr && sqdist != nullptr, "outputs are NULL");
    got = rbq::server_collect(srv, ticket, ids, sqdist, timeout_us, nullptr, latency_ns);
    if (!got) g_err = "timed out";
  });
  return g != RBQ_OK ? g : (got ? RBQ_OK : RBQ_EAGAIN);
}

rbq_status rbq_server_get_stats(rbq_server* srv, rbq_server_stats* st) {
  return guarded([&] {
    RBQ_CHECK(srv != nullptr && st != nullptr, "an argument is NULL");
    rbq::server_stats(srv, st);
  });
}

rbq_status rbq_server_destroy(rbq_server* srv) {
  return guarded([&] {
    RBQ_CHECK(srv != nullptr, "server is NULL");
    rbq::server_destroy(srv);
  });
}

rbq_status rbq_server_replay(rbq_server* srv, const rbq_replay_io* io) {
  return guarded([&] {
    RBQ_CHECK(srv != nullptr && io != nullptr, "an argument is NULL");
    rbq::server_replay(srv, *io);
  });
}

rbq_status rbq_replay_plain(rbq_index* idx, const rbq_replay_io* io) {
  return guarded([&] {
    RBQ_CHECK(idx != nullptr && io != nullptr, "an argument is NULL");
    rbq::replay_plain(idx, *io);
  });
}

const char* rbq_last_error(void) { return g_err.c_str(); }

const char* rbq_version(void) { return "librbq 0.1 (gfx950)"; }

}  // extern "C"
