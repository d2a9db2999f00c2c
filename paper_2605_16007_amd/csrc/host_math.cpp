#include "host_math.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <thread>
#include <unordered_set>

namespace rbq {

static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }

Rng::Rng(uint64_t seed) {
  uint64_t x = seed;
  for (auto& s : s_) s = splitmix64(x);
}

uint64_t Rng::next() {
  const uint64_t result = rotl(s_[1] * 5, 7) * 9;
  const uint64_t t = s_[1] << 17;
  s_[2] ^= s_[0];
  s_[3] ^= s_[1];
  s_[1] ^= s_[2];
  s_[0] ^= s_[3];
  s_[2] ^= t;
  s_[3] = rotl(s_[3], 45);
  return result;
}

double Rng::uniform() { return (next() >> 11) * 0x1.0p-53; }

double Rng::normal() {
  if (have_spare_) {
    have_spare_ = false;
    return spare_;
  }
  double u, v, s;
  do {
    u = 2.0 * uniform() - 1.0;
    v = 2.0 * uniform() - 1.0;
    s = u * u + v * v;
  } while (s >= 1.0 || s == 0.0);
  const double m = std::sqrt(-2.0 * std::log(s) / s);
  spare_ = v * m;
  have_spare_ = true;
  return u * m;
}

uint64_t Rng::below(uint64_t n) {
  // Lemire's nearly-divisionless bounded draw
  __uint128_t m = (__uint128_t)next() * n;
  uint64_t l = (uint64_t)m;
  if (l < n) {
    const uint64_t t = (0 - n) % n;
    while (l < t) {
      m = (__uint128_t)next() * n;
      l = (uint64_t)m;
    }
  }
  return (uint64_t)(m >> 64);
}

std::vector<double> haar_orthogonal(int d, Rng& rng) {
  // A = G (column-major working copy), Householder QR: A = Q R.
  std::vector<double> A((size_t)d * d);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) A[(size_t)j * d + i] = rng.normal();  // column j, row i
  std::vector<double> vs((size_t)d * d, 0.0), rdiag(d);
  for (int k = 0; k < d; ++k) {
    double* a = &A[(size_t)k * d];
    double norm = 0.0;
    for (int i = k; i < d; ++i) norm += a[i] * a[i];
    norm = std::sqrt(norm);
    const double alpha = a[k] > 0 ? -norm : norm;  // R_kk
    double* v = &vs[(size_t)k * d];
    for (int i = k; i < d; ++i) v[i] = a[i];
    v[k] -= alpha;
    double vn = 0.0;
    for (int i = k; i < d; ++i) vn += v[i] * v[i];
    rdiag[k] = alpha;
    if (vn > 0) {
      for (int j = k; j < d; ++j) {  // apply H = I - 2 v v^T / (v^T v) to columns k..d-1
        double* c = &A[(size_t)j * d];
        double dot = 0.0;
        for (int i = k; i < d; ++i) dot += v[i] * c[i];
        const double f = 2.0 * dot / vn;
        for (int i = k; i < d; ++i) c[i] -= f * v[i];
      }
      const double s = std::sqrt(vn);
      for (int i = k; i < d; ++i) v[i] /= s;  // unit v, H = I - 2 v v^T
    } else {
      for (int i = k; i < d; ++i) v[i] = 0.0;
    }
  }
  // Q = H_0 H_1 ... H_{d-1} applied to I (column-major), then Q diag(sign(R_kk)).
  std::vector<double> Q((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) Q[(size_t)i * d + i] = 1.0;
  for (int k = d - 1; k >= 0; --k) {
    const double* v = &vs[(size_t)k * d];
    for (int j = 0; j < d; ++j) {
      double* c = &Q[(size_t)j * d];
      double dot = 0.0;
      for (int i = k; i < d; ++i) dot += v[i] * c[i];
      for (int i = k; i < d; ++i) c[i] -= 2.0 * dot * v[i];
    }
  }
  std::vector<double> P((size_t)d * d);
  for (int j = 0; j < d; ++j) {
    const double sg = rdiag[j] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < d; ++i) P[(size_t)i * d + j] = Q[(size_t)j * d + i] * sg;  // row-major
  }
  return P;
}

std::vector<int64_t> sample_without_replacement(int64_t n, int64_t count, Rng& rng) {
  std::vector<int64_t> out;
  if (count >= n) {
    out.resize(n);
    std::iota(out.begin(), out.end(), 0);
    return out;
  }
  // Floyd's algorithm: exactly `count` draws, distinct results.
  std::unordered_set<int64_t> chosen;
  chosen.reserve((size_t)count * 2);
  for (int64_t j = n - count; j < n; ++j) {
    const int64_t t = (int64_t)rng.below((uint64_t)j + 1);
    if (!chosen.insert(t).second) chosen.insert(j);
  }
  out.assign(chosen.begin(), chosen.end());
  std::sort(out.begin(), out.end());
  return out;
}

void lloyd_update(const float* T, int64_t rows, int d, int ld, const int32_t* assign,
                  const double* dist, int nlist, float* C) {
  constexpr int CH = 16;
  std::vector<std::vector<double>> sums(CH);
  std::vector<std::vector<int64_t>> cnts(CH);
  const int64_t per = (rows + CH - 1) / CH;
  std::vector<std::thread> th;
  for (int c = 0; c < CH; ++c) {
    th.emplace_back([&, c] {
      auto& s = sums[c];
      auto& n = cnts[c];
      s.assign((size_t)nlist * d, 0.0);
      n.assign(nlist, 0);
      const int64_t r0 = c * per, r1 = std::min(rows, r0 + per);
      for (int64_t r = r0; r < r1; ++r) {
        const int j = assign[r];
        double* dst = &s[(size_t)j * d];
        const float* src = T + r * ld;
        for (int t = 0; t < d; ++t) dst[t] += src[t];
        ++n[j];
      }
    });
  }
  for (auto& t : th) t.join();
  std::vector<int> empty;
  for (int j = 0; j < nlist; ++j) {
    int64_t cnt = 0;
    for (int c = 0; c < CH; ++c) cnt += cnts[c][j];
    if (cnt == 0) {
      empty.push_back(j);
      continue;
    }
    for (int t = 0; t < d; ++t) {
      double acc = 0.0;
      for (int c = 0; c < CH; ++c) acc += sums[c][(size_t)j * d + t];
      C[(size_t)j * ld + t] = (float)(acc / (double)cnt);
    }
  }
  if (!empty.empty()) {
    std::vector<int64_t> order(rows);
    std::iota(order.begin(), order.end(), 0);
    const size_t m = std::min(empty.size(), (size_t)rows);
    std::partial_sort(order.begin(), order.begin() + m, order.end(), [&](int64_t a, int64_t b) {
      return dist[a] > dist[b] || (dist[a] == dist[b] && a < b);
    });
    for (size_t e = 0; e < m; ++e)
      for (int t = 0; t < d; ++t) C[(size_t)empty[e] * ld + t] = T[order[e] * ld + t];
  }
}

}  // namespace rbq
