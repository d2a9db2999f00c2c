// Host-side numerics of index construction: the library's own seeded random
// draws, a Haar-random orthogonal matrix, and the k-means centroid update.
#pragma once
#include <cstdint>
#include <vector>

namespace rbq {

// xoshiro256** seeded through splitmix64 (Blackman & Vigna). Deterministic
// across platforms; used for the library's own draws (P, k-means sampling).
class Rng {
 public:
  explicit Rng(uint64_t seed);
  uint64_t next();
  double uniform();          // [0, 1) with 53 random bits
  double normal();           // standard normal, Marsaglia polar method
  uint64_t below(uint64_t n);  // uniform integer in [0, n)
 private:
  uint64_t s_[4];
  bool have_spare_ = false;
  double spare_ = 0.0;
};

// Haar-random d x d orthogonal matrix (row-major, FP64): Householder QR of a
// Gaussian matrix with the signs of R's diagonal folded into Q.
std::vector<double> haar_orthogonal(int d, Rng& rng);

// `count` distinct indices of [0, n), ascending.
std::vector<int64_t> sample_without_replacement(int64_t n, int64_t count, Rng& rng);

// Lloyd update in FP64: each centroid becomes the mean of the rows assigned to
// it; an empty cluster moves to the row farthest from its centroid (distinct
// rows, farthest first). T is rows x ld (first d columns used), C nlist x ld.
// Sums run over 16 fixed row chunks so the result does not depend on the
// number of host threads.
void lloyd_update(const float* T, int64_t rows, int d, int ld, const int32_t* assign,
                  const double* dist, int nlist, float* C);

}  // namespace rbq
