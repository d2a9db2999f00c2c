// HIP kernels of librbq for gfx950 (CDNA4, wave64).
//
// Search path (Sec. 3.1.2): probe GEMM + top-nprobe (Phase 1), query rotation
// GEMM, B_q-bit query quantisation, 1-bit code scan with the estimator fused
// (Phase 3; Eqs. rabitq-ip-estimator, approx-dist), per-query top-R selection
// (Phase 4) and exact re-rank (Phase 5). Build path (Sec. 3.1.1): k-means
// assignment GEMM with fused argmin and the RaBitQ encoder (Phase 3).
#include <algorithm>
#include <mutex>
#include <cfloat>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace rbq {

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

__device__ inline uint32_t lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

__device__ inline float wave_sum(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ inline float wave_min(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off));
  return v;
}
__device__ inline float wave_max(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  return v;
}
__device__ inline int wave_sum_i(int v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Ascending bitonic sort of n (power of two) 64-bit keys in LDS by the whole
// workgroup. Ends with a barrier.
__device__ void bitonic_sort_lds(uint64_t* a, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n >> 1); t += blockDim.x) {
        const int i = 2 * t - (t & (stride - 1));
        const int j = i + stride;
        const uint64_t x = a[i], y = a[j];
        const bool up = (i & size) == 0;
        if ((x > y) == up) {
          a[i] = y;
          a[j] = x;
        }
      }
      __syncthreads();
    }
  }
}

// Inclusive prefix sum over a 256-thread workgroup. wsum: 4 words of LDS.
__device__ uint32_t block_incl_scan_256(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off);
    if (lane >= off) v += t;
  }
  if (lane == 63) wsum[wave] = v;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wave; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

}  // namespace

// ---------------------------------------------------------------------------
// FP32 GEMM on MFMA (v_mfma_f32_16x16x4f32). 64x64 block tile, K step 16,
// four waves of 32x32. Lane layout: A(i,k) in lane i+16k, B(k,j) in lane
// j+16k, result (i,j) in lane j+16*(i/4), register i%4.
// ---------------------------------------------------------------------------

__device__ inline void gemm_tile_load(const float* __restrict__ A, int lda, const float* __restrict__ B,
                                      int ldb, int M, int N, int K, int m0, int n0, int k0,
                                      float (*As)[17], float (*Bs)[17]) {
  const int tid = threadIdx.x;
  const int lr = tid >> 2, lc = (tid & 3) * 4;
  float4 av = make_float4(0.f, 0.f, 0.f, 0.f), bv = av;
  const int gk = k0 + lc;
  if (m0 + lr < M && gk < K) av = *reinterpret_cast<const float4*>(A + (size_t)(m0 + lr) * lda + gk);
  if (n0 + lr < N && gk < K) bv = *reinterpret_cast<const float4*>(B + (size_t)(n0 + lr) * ldb + gk);
  __syncthreads();
  As[lr][lc + 0] = av.x; As[lr][lc + 1] = av.y; As[lr][lc + 2] = av.z; As[lr][lc + 3] = av.w;
  Bs[lr][lc + 0] = bv.x; Bs[lr][lc + 1] = bv.y; Bs[lr][lc + 2] = bv.z; Bs[lr][lc + 3] = bv.w;
  __syncthreads();
}

__device__ inline void gemm_tile_mma(float (*As)[17], float (*Bs)[17], int wm, int wn, v4f (&acc)[2][2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int kk = s * 4 + (lane >> 4);
    const float a0 = As[wm + (lane & 15)][kk], a1 = As[wm + 16 + (lane & 15)][kk];
    const float b0 = Bs[wn + (lane & 15)][kk], b1 = Bs[wn + 16 + (lane & 15)][kk];
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b1, acc[1][1], 0, 0, 0);
  }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_gemm_tn(const float* __restrict__ A, int lda,
                                                 const float* __restrict__ B, int ldb,
                                                 float* __restrict__ C, int ldc, int M, int N, int K,
                                                 const float* __restrict__ bnorm) {
  __shared__ float As[64][17];
  __shared__ float Bs[64][17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  v4f acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    gemm_tile_load(A, lda, B, ldb, M, N, K, m0, n0, k0, As, Bs);
    gemm_tile_mma(As, Bs, wm, wn, acc);
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + ti * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + tj * 16 + (lane & 15);
        if (row < M && col < N) {
          float v = acc[ti][tj][r];
          if (MODE == 1) v = bnorm[col] - 2.0f * v;
          C[(size_t)row * ldc + col] = v;
        }
      }
}

void launch_gemm_tn(hipStream_t s, int mode, const float* A, int lda, const float* B, int ldb,
                    float* C, int ldc, int M, int N, int K, const float* bnorm) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  if (mode == 0)
    hipLaunchKernelGGL(k_gemm_tn<0>, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, bnorm);
  else
    hipLaunchKernelGGL(k_gemm_tn<1>, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K, bnorm);
  RBQ_HIP(hipGetLastError());
}

// Same product with BF16 inputs and FP32 accumulation
// (v_mfma_f32_16x16x16_bf16): each lane rounds its four A and four B values of
// a 16-deep K step to bfloat16 (nearest, ties to even) as it feeds the MFMA.
// Products of bfloat16 values are exact in FP32, so the result differs from the
// FP32 product only by the input rounding.
typedef short v4s __attribute__((ext_vector_type(4)));

__device__ inline short bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // finite inputs: round the low 16 bits away, ties to even
  return (short)(u >> 16);
}

__global__ __launch_bounds__(256) void k_gemm_tn_bf16(const float* __restrict__ A, int lda,
                                                      const float* __restrict__ B, int ldb,
                                                      float* __restrict__ C, int ldc, int M, int N,
                                                      int K) {
  __shared__ float As[64][17];
  __shared__ float Bs[64][17];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  const int r16 = lane & 15, kq = 4 * (lane >> 4);
  v4f acc[2][2];
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    gemm_tile_load(A, lda, B, ldb, M, N, K, m0, n0, k0, As, Bs);
    v4s a0, a1, b0, b1;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      a0[t] = bf16_rne(As[wm + r16][kq + t]);
      a1[t] = bf16_rne(As[wm + 16 + r16][kq + t]);
      b0[t] = bf16_rne(Bs[wn + r16][kq + t]);
      b1[t] = bf16_rne(Bs[wn + 16 + r16][kq + t]);
    }
    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b1, acc[1][1], 0, 0, 0);
  }
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + ti * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn + tj * 16 + (lane & 15);
        if (row < M && col < N) C[(size_t)row * ldc + col] = acc[ti][tj][r];
      }
}

void launch_gemm_tn_bf16(hipStream_t s, const float* A, int lda, const float* B, int ldb, float* C,
                         int ldc, int M, int N, int K) {
  if (M <= 0 || N <= 0) return;
  dim3 grid((N + 63) / 64, (M + 63) / 64);
  hipLaunchKernelGGL(k_gemm_tn_bf16, grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, M, N, K);
  RBQ_HIP(hipGetLastError());
}

// Nearest centroid per row: each workgroup owns 64 rows of A and walks every
// 64-column tile of B, keeping the running minimum of key64(score, column).
__global__ __launch_bounds__(256) void k_assign_argmin(const float* __restrict__ A, int lda,
                                                       const float* __restrict__ B, int ldb,
                                                       const float* __restrict__ bnorm, int M, int N,
                                                       int K, uint64_t* __restrict__ out) {
  __shared__ float As[64][17];
  __shared__ float Bs[64][17];
  __shared__ unsigned long long best[64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.x * 64;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  if (tid < 64) best[tid] = KEY_NONE;
  __syncthreads();
  for (int n0 = 0; n0 < N; n0 += 64) {
    v4f acc[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
      gemm_tile_load(A, lda, B, ldb, M, N, K, m0, n0, k0, As, Bs);
      gemm_tile_mma(As, Bs, wm, wn, acc);
    }
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wm + ti * 16 + 4 * (lane >> 4) + r;
        unsigned long long kb = KEY_NONE;
#pragma unroll
        for (int tj = 0; tj < 2; ++tj) {
          const int col = n0 + wn + tj * 16 + (lane & 15);
          if (col < N) {
            const unsigned long long kk = key64(bnorm[col] - 2.0f * acc[ti][tj][r], (uint32_t)col);
            kb = kk < kb ? kk : kb;
          }
        }
        for (int off = 1; off < 16; off <<= 1) {
          const unsigned long long o = __shfl_xor(kb, off);
          kb = o < kb ? o : kb;
        }
        if ((lane & 15) == 0) atomicMin(&best[rl], kb);
      }
  }
  __syncthreads();
  if (tid < 64 && m0 + tid < M) out[m0 + tid] = best[tid];
}

void launch_assign_argmin(hipStream_t s, const float* A, int lda, const float* B, int ldb,
                          const float* bnorm, int M, int N, int K, uint64_t* out) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_assign_argmin, dim3((M + 63) / 64), dim3(256), 0, s, A, lda, B, ldb, bnorm,
                     M, N, K, out);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Row top-k: exact selection of the k smallest 64-bit keys of each row by an
// MSB-first radix select, compaction, and (sorted mode) an LDS bitonic sort of
// the k survivors. The row is staged in LDS when it fits (up to ~150 KB). The
// digits start at the highest bit in which the row's smallest and largest keys
// differ (bits above it are common to every key and would only pile every
// histogram atomic onto one bin); each pass takes up to 8 bits and the select
// stops as soon as the boundary bucket is taken whole. Compaction appends with
// one LDS atomic per wave (ballot + lane prefix).
// ---------------------------------------------------------------------------

// Inclusive prefix sum of hist[0..256) for a workgroup of NT threads
// (threads >= 256 contribute 0). wsum: 4 words of LDS.
template <int NT>
__device__ uint32_t hist_incl_scan(uint32_t v, uint32_t* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off);
    if (lane >= off) v += t;
  }
  if (lane == 63 && wave < 4) wsum[wave] = v;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wave && w < 4; ++w) add += wsum[w];
  __syncthreads();
  return v + add;
}

template <bool FROM_SCORE, int NT>
__global__ __launch_bounds__(NT) void k_row_topk(TopkArgs a) {
  constexpr int NW = NT / 64;       // waves
  constexpr int NH = NT >= 512 ? 4 : 1;  // histogram copies (waves share copy w % NH)
  extern __shared__ uint64_t smem[];
  __shared__ uint32_t hist[NH][256];
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t s_digit, s_rem, s_bucket, s_cnt;
  __shared__ uint64_t s_lo[NW], s_hi[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row = blockIdx.x;
  const int k = a.rowk ? a.rowk[row] : a.k, KP = a.KP;
  int ncols = a.ncols;
  if (a.rowcnt) {  // pool mode: the row holds a.k running keys then rowcnt[row] new ones
    const uint32_t extra = min(a.rowcnt[row], (uint32_t)a.max_extra);
    if (extra == 0) return;
    ncols = a.k + (int)extra;
  }
  const bool cached = ncols <= a.cache_cap;
  uint64_t* cache = smem;
  // selection buffer: after the cache (sorted mode); for unsorted output a
  // cached row is compacted straight into the output row (all of its reads
  // come from the cache), and an uncached row uses the cache space instead
  const bool direct = !a.sorted && cached && a.out_keys && !a.out_low && !a.out_val;
  uint64_t* sel = a.sorted ? smem + a.cache_cap : smem;
  uint64_t* dst = direct ? a.out_keys + row * a.ldo : sel;
  auto src = [&](int c) -> uint64_t {
    if (FROM_SCORE) return key64(a.score[row * a.ld + c], (uint32_t)c);
    return a.keys[row * a.ld + c];
  };
  auto get = [&](int c) -> uint64_t { return cached ? cache[c] : src(c); };

  const bool take_all = ncols <= k;
  uint64_t prefix = 0, pmask = 0;
  uint32_t rem = (uint32_t)k;
  {
    // stage the row (eight loads in flight per thread); smallest and largest key
    uint64_t lo = ~0ull, hi = 0;
    for (int c0 = 0; c0 < ncols; c0 += 8 * NT) {
      uint64_t v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * NT + tid;
        v[u] = c < ncols ? src(c) : 0ull;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + u * NT + tid;
        if (c < ncols) {
          if (cached) cache[c] = v[u];
          lo = v[u] < lo ? v[u] : lo;
          hi = v[u] > hi ? v[u] : hi;
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
      lo = l2 < lo ? l2 : lo;
      hi = h2 > hi ? h2 : hi;
    }
    if (lane == 0) {
      s_lo[wave] = lo;
      s_hi[wave] = hi;
    }
    __syncthreads();
    lo = s_lo[0];
    hi = s_hi[0];
    for (int w = 1; w < NW; ++w) {
      lo = s_lo[w] < lo ? s_lo[w] : lo;
      hi = s_hi[w] > hi ? s_hi[w] : hi;
    }
    const uint64_t diff = lo ^ hi;
    const int top = diff ? 63 - __clzll((long long)diff) : -1;  // highest bit in which keys differ
    if (top < 63) {  // bits above `top` are the same in every key
      pmask = top < 0 ? ~0ull : ~((2ull << top) - 1ull);
      prefix = lo & pmask;
    }
    if (!take_all) {
      for (int hb = top; hb >= 0;) {
        const int lb = hb >= 7 ? hb - 7 : 0;
        const uint64_t dmask = ((2ull << (hb - lb)) - 1ull);
        for (int t = tid; t < NH * 256; t += NT) (&hist[0][0])[t] = 0;
        __syncthreads();
        uint32_t* hw = hist[wave % NH];
        for (int c = tid; c < ncols; c += NT) {
          const uint64_t key = get(c);
          if ((key & pmask) == prefix) atomicAdd(&hw[(key >> lb) & dmask], 1u);
        }
        __syncthreads();
        uint32_t h = 0;
        if (tid < 256)
          for (int t = 0; t < NH; ++t) h += hist[t][tid];
        const uint32_t incl = hist_incl_scan<NT>(h, wsum);
        const uint32_t excl = incl - h;
        if (tid < 256 && excl < rem && rem <= incl) {
          s_digit = (uint32_t)tid;
          s_rem = rem - excl;
          s_bucket = h;
        }
        __syncthreads();
        prefix |= (uint64_t)s_digit << lb;
        pmask |= dmask << lb;
        rem = s_rem;
        const uint32_t bucket = s_bucket;
        __syncthreads();
        if (bucket == rem) break;
        hb = lb - 1;
      }
    }
  }
  if (tid == 0) s_cnt = 0;
  __syncthreads();
  // compaction: keys below the prefix, then boundary-bucket keys up to k in all
  const int rounds = (ncols + NT - 1) / NT;
  uint64_t mx = 0;  // the largest key this thread wrote
  if (take_all) {
    for (int r = 0; r < rounds; ++r) {
      const int c = r * NT + tid;
      const bool t = c < ncols;
      const uint64_t m = __ballot(t);
      uint32_t base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
      base = __shfl(base, 0);
      if (t) {
        const uint64_t key = get(c);
        dst[base + lane_prefix(m)] = key;
        mx = key > mx ? key : mx;
      }
    }
  } else {
    const uint64_t hi_key = prefix | ~pmask;
    for (int r = 0; r < rounds; ++r) {
      const int c = r * NT + tid;
      const uint64_t key = c < ncols ? get(c) : KEY_NONE;
      const bool t = c < ncols && key < prefix;
      const uint64_t m = __ballot(t);
      uint32_t base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
      base = __shfl(base, 0);
      if (t) {
        dst[base + lane_prefix(m)] = key;
        mx = key > mx ? key : mx;
      }
    }
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
      const int c = r * NT + tid;
      const uint64_t key = c < ncols ? get(c) : KEY_NONE;
      const bool t = c < ncols && key >= prefix && key <= hi_key;
      const uint64_t m = __ballot(t);
      uint32_t base = 0;
      if (lane == 0 && m) base = atomicAdd(&s_cnt, (uint32_t)__popcll(m));
      base = __shfl(base, 0);
      const uint32_t p = base + lane_prefix(m);
      if (t && p < (uint32_t)k) {
        dst[p] = key;
        mx = key > mx ? key : mx;
      }
    }
  }
  __syncthreads();
  const int cnt = min((int)s_cnt, k);
  const int fill_to = a.sorted ? KP : k;
  for (int i = cnt + tid; i < fill_to; i += NT) dst[i] = KEY_NONE;
  __syncthreads();
  uint64_t kth;  // the k-th smallest key (KEY_NONE if fewer than k)
  if (a.sorted) {
    bitonic_sort_lds(sel, KP);
    kth = sel[k - 1];
  } else {  // the selected keys in any order; their maximum is the k-th
    for (int off = 32; off > 0; off >>= 1) {
      const uint64_t o = __shfl_xor(mx, off);
      mx = o > mx ? o : mx;
    }
    if (lane == 0) s_hi[wave] = mx;
    __syncthreads();
    kth = s_hi[0];
    for (int w = 1; w < NW; ++w) kth = s_hi[w] > kth ? s_hi[w] : kth;
    if (cnt < k) kth = KEY_NONE;  // fewer than k keys
  }
  for (int i = tid; i < k && !direct; i += NT) {
    const uint64_t v = sel[i];
    if (a.out_keys) a.out_keys[row * a.ldo + i] = v;
    if (a.out_low) a.out_low[row * k + i] = v == KEY_NONE ? -1 : (int32_t)(uint32_t)v;
    if (a.out_val) a.out_val[row * k + i] = v == KEY_NONE ? INFINITY : f32_ord((uint32_t)(v >> 32));
  }
  if (tid == 0) {
    if (a.rowcnt) a.rowcnt[row] = 0;
    if (a.qthr && kth != KEY_NONE) atomicMin(&a.qthr[row], (uint32_t)(kth >> 32));
  }
}

// ---------------------------------------------------------------------------
// Pool merge: the same selection for a query's candidate row in pool mode
// (k running keys, then rowcnt[row] new ones; the k smallest are written, in
// any order, to the row's first k slots). The row is held in registers, KPT
// keys per thread, in pieces of NT * KPT keys (one piece for rows up to that
// size, read once; larger rows are re-read per pass, and the first piece,
// which holds the output slots, is always read before any write). Histogram
// counts are fire-and-forget LDS atomics; the output positions come from one
// workgroup scan per piece (keys below the boundary digit, then boundary keys
// up to k). Small LDS and registers: two workgroups per CU.
// ---------------------------------------------------------------------------

// Exclusive scan of v over a workgroup of NT threads; *total = the sum.
// wsum: NT/64 words of LDS.
template <int NT>
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* wsum, uint32_t* total) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(x, off);
    if (lane >= off) x += t;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = wsum[w];
    before += w < wave ? t : 0u;
    all += t;
  }
  __syncthreads();
  *total = all;
  return before + x - v;
}

// Output rows of up to this many keys are assembled in LDS and then copied
// out with consecutive threads on consecutive keys (the compaction's own
// stores go to scattered positions).
constexpr int kMergeStageKeys = 4096;

template <int NT, int KPT>
__global__ __launch_bounds__(NT) void k_pool_merge(TopkArgs a) {
  constexpr int NW = NT / 64;
  extern __shared__ uint64_t s_out[];  // a.k keys when a.k <= kMergeStageKeys
  constexpr int NH = 4;  // histogram copies (wave w uses copy w % NH)
  constexpr int PIECE = NT * KPT;
  __shared__ uint32_t hist[NH][256];
  __shared__ uint32_t wsum[NW > 4 ? NW : 4];
  __shared__ uint32_t s_digit, s_rem, s_bucket;
  __shared__ uint64_t s_lo[NW], s_hi[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row = blockIdx.x;
  const uint32_t extra = min(a.rowcnt[row], (uint32_t)a.max_extra);
  if (extra == 0) return;
  const int k = a.rowk ? a.rowk[row] : a.k;
  const int ncols = a.k + (int)extra;
  const uint64_t* src = a.keys + row * a.ld;
  uint64_t* const out = a.out_keys + row * a.ldo;
  const bool staged = a.k <= kMergeStageKeys;
  uint64_t* dst = staged ? s_out : out;
  const bool one = ncols <= PIECE;
  uint64_t v[KPT];
  auto load = [&](int p0) {
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
      const int c = p0 + u * NT + tid;
      v[u] = c < ncols ? src[c] : KEY_NONE;
    }
  };
  // (slots past ncols read as KEY_NONE and are never counted or written:
  // every count below is over c < ncols)
  auto valid = [&](int p0, int u) { return p0 + u * NT + tid < ncols; };

  // smallest and largest key
  uint64_t lo = ~0ull, hi = 0;
  for (int p0 = 0; p0 < ncols; p0 += PIECE) {
    load(p0);
#pragma unroll
    for (int u = 0; u < KPT; ++u)
      if (valid(p0, u)) {
        lo = v[u] < lo ? v[u] : lo;
        hi = v[u] > hi ? v[u] : hi;
      }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  if (lane == 0) {
    s_lo[wave] = lo;
    s_hi[wave] = hi;
  }
  __syncthreads();
  lo = s_lo[0];
  hi = s_hi[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    lo = s_lo[w] < lo ? s_lo[w] : lo;
    hi = s_hi[w] > hi ? s_hi[w] : hi;
  }
  // MSB-first radix select from the highest bit in which the keys differ
  uint64_t prefix = 0, pmask = 0;
  uint32_t rem = (uint32_t)k;
  const uint64_t diff = lo ^ hi;
  const int top = diff ? 63 - __clzll((long long)diff) : -1;
  if (top < 63) {
    pmask = top < 0 ? ~0ull : ~((2ull << top) - 1ull);
    prefix = lo & pmask;
  }
  for (int hb = top; hb >= 0;) {
    const int lb = hb >= 7 ? hb - 7 : 0;
    const uint64_t dmask = (2ull << (hb - lb)) - 1ull;
    for (int t = tid; t < NH * 256; t += NT) (&hist[0][0])[t] = 0u;
    __syncthreads();
    uint32_t* hw = hist[wave % NH];
    for (int p0 = 0; p0 < ncols; p0 += PIECE) {
      if (!one) load(p0);
#pragma unroll
      for (int u = 0; u < KPT; ++u)
        if (valid(p0, u) && (v[u] & pmask) == prefix) atomicAdd(&hw[(v[u] >> lb) & dmask], 1u);
    }
    __syncthreads();
    uint32_t h = 0;
    if (tid < 256)
#pragma unroll
      for (int t = 0; t < NH; ++t) h += hist[t][tid];
    const uint32_t incl = hist_incl_scan<NT>(h, wsum);
    const uint32_t excl = incl - h;
    if (tid < 256 && excl < rem && rem <= incl) {
      s_digit = (uint32_t)tid;
      s_rem = rem - excl;
      s_bucket = h;
    }
    __syncthreads();
    prefix |= (uint64_t)s_digit << lb;
    pmask |= dmask << lb;
    rem = s_rem;
    const uint32_t bucket = s_bucket;
    __syncthreads();
    if (bucket == rem) break;
    hb = lb - 1;
  }
  // compaction: keys below the boundary bucket fill [0, k - rem); boundary
  // keys fill [k - rem, k) in arrival order until rem are taken
  const uint64_t hi_key = prefix | ~pmask;
  const uint32_t nlt = (uint32_t)k - rem;
  uint32_t base_lt = 0, base_eq = 0;
  uint64_t mx = 0;
  if (!one) load(0);  // the first piece holds every output slot: read before any write
  __syncthreads();
  for (int p0 = 0; p0 < ncols; p0 += PIECE) {
    if (!one && p0 > 0) load(p0);
    uint32_t clt = 0, ceq = 0;
#pragma unroll
    for (int u = 0; u < KPT; ++u)
      if (valid(p0, u)) {
        clt += v[u] < prefix ? 1u : 0u;
        ceq += (v[u] >= prefix && v[u] <= hi_key) ? 1u : 0u;
      }
    uint32_t tot;
    const uint32_t ex = block_excl_scan<NT>((clt << 16) | ceq, wsum, &tot);
    uint32_t plt = base_lt + (ex >> 16), peq = base_eq + (ex & 0xFFFFu);
#pragma unroll
    for (int u = 0; u < KPT; ++u)
      if (valid(p0, u)) {
        if (v[u] < prefix) {
          dst[plt++] = v[u];
          mx = v[u] > mx ? v[u] : mx;
        } else if (v[u] <= hi_key) {
          if (peq < rem) {
            dst[nlt + peq] = v[u];
            mx = v[u] > mx ? v[u] : mx;
          }
          ++peq;
        }
      }
    base_lt += tot >> 16;
    base_eq += tot & 0xFFFFu;
  }
  // the k-th smallest key is the largest one written
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if (lane == 0) s_hi[wave] = mx;
  __syncthreads();
  if (staged)
    for (int i = tid; i < k; i += NT) out[i] = s_out[i];
  if (tid == 0) {
    uint64_t kth = s_hi[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) kth = s_hi[w] > kth ? s_hi[w] : kth;
    a.rowcnt[row] = 0;
    if (a.qthr && kth != KEY_NONE) atomicMin(&a.qthr[row], (uint32_t)(kth >> 32));
  }
}

static int pow2_at_least(int n) {
  int p = 2;
  while (p < n) p <<= 1;
  return p;
}

constexpr size_t kTopkLdsMax = 150u << 10;  // dynamic LDS of one selection workgroup

// Sorted top-k of float scores with the row in registers (rows of up to
// kScoreTopkCols scores: 16 per thread, 256 threads up to 4096 columns, 512
// above); defined with the register-resident selection. Longer rows stream
// past a bound set by their first kScoreTopkCols scores.
constexpr int kScoreTopkCols = 512 * 16;
static void launch_score_topk(hipStream_t s, const TopkArgs& a, int rows);
static void launch_score_topk_long(hipStream_t s, const TopkArgs& a, int rows);

void launch_row_topk(hipStream_t s, TopkArgs a, int rows) {
  if (rows <= 0) return;
  RBQ_CHECK(a.k >= 1 && a.k <= MAX_SEL, "selection size out of range");
  a.KP = pow2_at_least(a.k);
  if (a.ldo <= 0) a.ldo = a.k;
  const int maxcols = a.rowcnt ? a.k + a.max_extra : a.ncols;
  // sorted mode: the row cache, then a KP-key selection buffer; unsorted
  // mode: the cache alone (a cached row is compacted into its output row, an
  // uncached one into the cache space, which then holds at least k keys)
  const int slots = (int)(kTopkLdsMax / sizeof(uint64_t));
  int lds_keys;
  if (a.sorted) {
    a.cache_cap = std::max(0, std::min(maxcols, slots - a.KP));
    lds_keys = a.cache_cap + a.KP;
  } else {
    RBQ_CHECK(a.out_keys && !a.out_low && !a.out_val, "unsorted selection writes keys only");
    a.cache_cap = std::min(maxcols, slots);
    lds_keys = std::max(a.cache_cap, a.k);
  }
  const size_t lds = (size_t)lds_keys * sizeof(uint64_t);
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    for (const void* f : {reinterpret_cast<const void*>(k_row_topk<true, 256>),
                          reinterpret_cast<const void*>(k_row_topk<false, 256>),
                          reinterpret_cast<const void*>(k_row_topk<false, 1024>)})
      RBQ_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kTopkLdsMax));
  });
  // pool merges: the register-resident kernel
  if (a.rowcnt && !a.sorted) {
    // (a row longer than one piece of NT x 32 keys is merged piece by piece)
    const int nt = a.merge_threads == 256 ? 256 : 512;
    RBQ_CHECK(a.k <= nt * 32, "pool merge: running keys exceed one piece");
    const size_t stage = a.k <= kMergeStageKeys ? (size_t)a.k * sizeof(uint64_t) : 0;
    if (nt == 256)
      hipLaunchKernelGGL((k_pool_merge<256, 32>), dim3(rows), dim3(256), stage, s, a);
    else
      hipLaunchKernelGGL((k_pool_merge<512, 32>), dim3(rows), dim3(512), stage, s, a);
    RBQ_HIP(hipGetLastError());
    return;
  }
  if (a.score && a.sorted && a.ncols <= kScoreTopkCols && !a.rowcnt) {
    launch_score_topk(s, a, rows);
    return;
  }
  if (a.score && a.sorted && !a.rowcnt && !a.rowk) {
    launch_score_topk_long(s, a, rows);
    return;
  }
  if (a.score)
    hipLaunchKernelGGL((k_row_topk<true, 256>), dim3(rows), dim3(256), lds, s, a);
  else if (a.rowcnt)
    hipLaunchKernelGGL((k_row_topk<false, 1024>), dim3(rows), dim3(1024), lds, s, a);
  else
    hipLaunchKernelGGL((k_row_topk<false, 256>), dim3(rows), dim3(256), lds, s, a);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Query quantisation: 16 lanes per (query, probe) pair, four pairs per wave;
// lane g of a pair holds 8 consecutive dimensions of every 128-dimension step.
// r = P^T q - P^T c_j, v_l = min r, Delta = (max r - v_l)/(2^bq - 1),
// qu = floor((r - v_l)/Delta + 1/2) clamped; ||r||^2 and sum qu. The qu bytes
// are stored 8 per lane, and bit-plane word w (dimensions 32w..32w+31) is
// assembled from the bytes of the four lanes that hold those dimensions.
// Workgroup (x, y) takes query x and probe ranks 16y..16y+15. The pair's
// reductions run on DPP lane moves inside its 16-lane row: rotations by 8 and
// 4, then swaps within quads by 2 and 1, which combine the same pairs in the
// same order as an xor butterfly over 8, 4, 2, 1, so lane 0's sum of squares
// is that butterfly's.
// ---------------------------------------------------------------------------

__device__ inline void load8(const float* p, int d0, int d, float (&v)[8]) {
  if (d0 + 8 <= d) {  // rows are 16-byte aligned and d0 is a multiple of 8
    const float4 a = *reinterpret_cast<const float4*>(p + d0);
    const float4 b = *reinterpret_cast<const float4*>(p + d0 + 4);
    v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
    v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
  } else {
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = d0 + u < d ? p[d0 + u] : 0.f;
  }
}

// the value of lane CTRL(lane) of this lane's row of 16 (DPP control CTRL)
template <int CTRL>
__device__ inline uint32_t dpp_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ inline float dpp_f32(float v) {
  return __uint_as_float(dpp_u32<CTRL>(__float_as_uint(v)));
}
constexpr int kDppRor8 = 0x128, kDppRor4 = 0x124;  // row rotations
constexpr int kDppXor2 = 0x4E, kDppXor1 = 0xB1;    // quad permutations [2,3,0,1], [1,0,3,2]

template <int STEPS, bool INJ>
__global__ __launch_bounds__(256) void k_quant(const float* __restrict__ qrot, int ldq,
                                               const float* __restrict__ crot, int ldc,
                                               const int32_t* __restrict__ probes, int nprobe, int d,
                                               int W, int bq, int bqs, uint32_t* __restrict__ planes,
                                               uint8_t* __restrict__ qu_out, uint8_t* __restrict__ qu8,
                                               int qu8_ld, float4* __restrict__ scal,
                                               const uint8_t* __restrict__ inj_qu,
                                               const float* __restrict__ inj_scal) {
  const int g = threadIdx.x & 15;
  const int64_t i = blockIdx.x;
  const int p = (int)blockIdx.y * 16 + (int)(threadIdx.x >> 4);
  const bool active = p < nprobe;  // (the 16 lanes of a pair agree)
  const int64_t pr = i * nprobe + (active ? p : 0);
  const int j = max(probes[pr], 0);  // -1 (not probed): computed on list 0 and never used
  const float* qr = qrot + i * ldq;
  const float* cr = crot + (int64_t)j * ldc;
  const int Wq = W * 32;
  const int steps = STEPS > 0 ? STEPS : (Wq + 127) / 128;
  float rmin = INFINITY, rmax = -INFINITY, ss = 0.f;
  float r0[8];  // the first step's residuals (all of them when d <= 128)
  for (int st = 0; st < steps; ++st) {
    const int d0 = st * 128 + 8 * g;
    float a[8], c[8];
    load8(qr, d0, d, a);
    load8(cr, d0, d, c);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const float r = a[u] - c[u];
      if (st == 0) r0[u] = r;
      if (d0 + u < d) {
        rmin = fminf(rmin, r);
        rmax = fmaxf(rmax, r);
        ss += r * r;
      }
    }
  }
  rmin = fminf(rmin, dpp_f32<kDppRor8>(rmin));
  rmax = fmaxf(rmax, dpp_f32<kDppRor8>(rmax));
  ss += dpp_f32<kDppRor8>(ss);
  rmin = fminf(rmin, dpp_f32<kDppRor4>(rmin));
  rmax = fmaxf(rmax, dpp_f32<kDppRor4>(rmax));
  ss += dpp_f32<kDppRor4>(ss);
  rmin = fminf(rmin, dpp_f32<kDppXor2>(rmin));
  rmax = fmaxf(rmax, dpp_f32<kDppXor2>(rmax));
  ss += dpp_f32<kDppXor2>(ss);
  rmin = fminf(rmin, dpp_f32<kDppXor1>(rmin));
  rmax = fmaxf(rmax, dpp_f32<kDppXor1>(rmax));
  ss += dpp_f32<kDppXor1>(ss);
  float vl, delta, rn2;
  if (INJ && inj_scal) {
    rn2 = inj_scal[pr * 3 + 0];
    vl = inj_scal[pr * 3 + 1];
    delta = inj_scal[pr * 3 + 2];
  } else {
    rn2 = ss;
    vl = rmin;
    delta = (rmax - rmin) / (float)((1 << bq) - 1);
  }
  const float inv = delta > 0.f ? 1.0f / delta : 0.f;
  const uint32_t top = (1u << bq) - 1u;
  int sq = 0;
  for (int st = 0; st < steps; ++st) {
    const int d0 = st * 128 + 8 * g;
    float r[8];
    if (st == 0) {
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = r0[u];
    } else {
      float a[8], c[8];
      load8(qr, d0, d, a);
      load8(cr, d0, d, c);
#pragma unroll
      for (int u = 0; u < 8; ++u) r[u] = a[u] - c[u];
    }
    uint32_t lo = 0, hi = 0;
    uint32_t qv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int dd = d0 + u;
      uint32_t q = 0;
      if (dd < d) {
        if (INJ && inj_qu) {
          q = inj_qu[pr * d + dd];
        } else {
          // f is integral and at least 0 (r >= v_l): clamping it to [0, top]
          // and truncating gives the code
          const float y = (r[u] - vl) * inv;
          const float f = floorf(y + 0.5f);
          q = (uint32_t)__builtin_amdgcn_fmed3f(f, 0.f, (float)top);
        }
      }
      sq += (int)q;
      qv[u] = q;
      if (u < 4)
        lo |= q << (8 * u);
      else
        hi |= q << (8 * (u - 4));
    }
    // plane word w (dimensions 32w..32w+31) from the bytes of lanes 4k..4k+3
    // of the pair (k = g / 4): lane 4k + t stores planes t and t + 4. Bit b
    // of each of four bytes is gathered by one multiply: the bits sit at 0,
    // 8, 16, 24 and x 0x10204080 moves them to 28..31 with no carries.
    const int t = g & 3;
    uint32_t wd[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      if (b >= bqs) {
        wd[b] = 0u;
        continue;
      }
      const uint32_t pl = (((lo >> b) & 0x01010101u) * 0x10204080u) >> 28;
      const uint32_t ph = (((hi >> b) & 0x01010101u) * 0x10204080u) >> 28;
      uint32_t v = (pl | (ph << 4)) << (8 * t);
      v |= dpp_u32<kDppXor1>(v);
      v |= dpp_u32<kDppXor2>(v);
      wd[b] = v;
    }
    if (qu8 && active) {  // every lane: the row's bytes past d are zeros
      // (the offsets of j = 1, 2, 3 are those of j = 0 plus 8, 32, 40)
      uint8_t* row = qu8 + pr * qu8_ld + st * 128 + group_qu8_offset(g, 0);
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int v = __builtin_amdgcn_cvt_pk_fp8_f32((float)(qv[j] << 1), (float)(qv[j + 4] << 1), 0, false);
        *reinterpret_cast<uint16_t*>(row + 32 * (j >> 1) + 8 * (j & 1)) = (uint16_t)v;
      }
    }
    if (active && d0 < Wq) {
      if (qu_out) *reinterpret_cast<uint2*>(qu_out + pr * Wq + d0) = make_uint2(lo, hi);
      const int w = d0 >> 5;
      uint32_t* pw = planes + (pr * W + w) * bqs;
      const uint32_t v0 = t == 0 ? wd[0] : t == 1 ? wd[1] : t == 2 ? wd[2] : wd[3];
      const uint32_t v1 = t == 0 ? wd[4] : t == 1 ? wd[5] : t == 2 ? wd[6] : wd[7];
      if (t < bqs) pw[t] = t < bq ? v0 : 0u;
      if (t + 4 < bqs) pw[t + 4] = t + 4 < bq ? v1 : 0u;
    }
  }
  sq += (int)dpp_u32<kDppRor8>((uint32_t)sq);
  sq += (int)dpp_u32<kDppRor4>((uint32_t)sq);
  sq += (int)dpp_u32<kDppXor2>((uint32_t)sq);
  sq += (int)dpp_u32<kDppXor1>((uint32_t)sq);
  if (active && g == 0) scal[pr] = make_float4(rn2, vl, delta, (float)sq);
}

void launch_quant(hipStream_t s, const float* qrot, int ldq, const float* crot, int ldc,
                  const int32_t* probes, int nq, int nprobe, int d, int W, int bq, int bqs,
                  uint32_t* planes, uint8_t* qu, uint8_t* qu8, int qu8_ld, float4* scal,
                  const uint8_t* inj_qu, const float* inj_scal) {
  if (nq <= 0 || nprobe <= 0) return;
  RBQ_CHECK(!qu8 || (bq <= 4 && qu8_ld == 128 * ((W * 32 + 127) / 128)), "quantisation: fp8 operand rows");
  RBQ_CHECK(bq >= 1 && bq <= 8 && bqs <= 8, "query bits out of range");
  RBQ_CHECK((nprobe + 15) / 16 <= 65535, "quantisation: nprobe out of range");
  const dim3 grid((unsigned)nq, (unsigned)((nprobe + 15) / 16));
  const int steps = (W * 32 + 127) / 128;
  const bool inj = inj_qu || inj_scal;
#define RBQ_QUANT(ST, INJV)                                                                            \
  hipLaunchKernelGGL((k_quant<ST, INJV>), grid, dim3(256), 0, s, qrot, ldq, crot, ldc, probes, nprobe, d, \
                     W, bq, bqs, planes, qu, qu8, qu8_ld, scal, inj_qu, inj_scal)
  if (inj)
    RBQ_QUANT(0, true);
  else if (steps == 1)
    RBQ_QUANT(1, false);
  else if (steps == 2)
    RBQ_QUANT(2, false);
  else
    RBQ_QUANT(0, false);
#undef RBQ_QUANT
  RBQ_HIP(hipGetLastError());
}

// LDS of a register-resident selection (select_regs) by NT threads.
template <int NT>
struct SelRegShared {
  uint32_t hist[4][256];
  uint32_t wsum[NT / 64 > 4 ? NT / 64 : 4];
  uint32_t digit, rem, bucket;
  uint64_t lo[NT / 64], hi[NT / 64];
};

// The k smallest of the n keys held KPT per thread (key u of thread t is key
// u * NT + t; keys at n and beyond are ignored) written to dst[0..k) in any
// order; returns the k-th smallest, or KEY_NONE when n <= k (then every key is
// written). Every thread must call it; the keys must not live in dst's range
// of memory except in these registers (all reads are done before the first
// write, behind a barrier). Ends with a barrier.
template <int NT, int KPT>
__device__ uint64_t select_regs(const uint64_t (&v)[KPT], int n, int k, uint64_t* dst, SelRegShared<NT>& sh) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  auto valid = [&](int u) { return u * NT + tid < n; };
  uint64_t lo = ~0ull, hi = 0;
#pragma unroll
  for (int u = 0; u < KPT; ++u)
    if (valid(u)) {
      lo = v[u] < lo ? v[u] : lo;
      hi = v[u] > hi ? v[u] : hi;
    }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  if (lane == 0) {
    sh.lo[wave] = lo;
    sh.hi[wave] = hi;
  }
  __syncthreads();
  lo = sh.lo[0];
  hi = sh.hi[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) {
    lo = sh.lo[w] < lo ? sh.lo[w] : lo;
    hi = sh.hi[w] > hi ? sh.hi[w] : hi;
  }
  const bool take_all = n <= k;
  uint64_t prefix = 0, pmask = 0;
  uint32_t rem = (uint32_t)(take_all ? n : k);
  if (!take_all) {
    const uint64_t diff = lo ^ hi;
    const int top = diff ? 63 - __clzll((long long)diff) : -1;
    if (top < 63) {
      pmask = top < 0 ? ~0ull : ~((2ull << top) - 1ull);
      prefix = lo & pmask;
    }
    for (int hb = top; hb >= 0;) {
      const int lb = hb >= 7 ? hb - 7 : 0;
      const uint64_t dmask = (2ull << (hb - lb)) - 1ull;
      for (int t = tid; t < 4 * 256; t += NT) (&sh.hist[0][0])[t] = 0u;
      __syncthreads();
      uint32_t* hw = sh.hist[wave & 3];
#pragma unroll
      for (int u = 0; u < KPT; ++u)
        if (valid(u) && (v[u] & pmask) == prefix) atomicAdd(&hw[(v[u] >> lb) & dmask], 1u);
      __syncthreads();
      uint32_t h = 0;
      if (tid < 256) h = sh.hist[0][tid] + sh.hist[1][tid] + sh.hist[2][tid] + sh.hist[3][tid];
      const uint32_t incl = hist_incl_scan<NT>(h, sh.wsum);
      const uint32_t excl = incl - h;
      if (tid < 256 && excl < rem && rem <= incl) {
        sh.digit = (uint32_t)tid;
        sh.rem = rem - excl;
        sh.bucket = h;
      }
      __syncthreads();
      prefix |= (uint64_t)sh.digit << lb;
      pmask |= dmask << lb;
      rem = sh.rem;
      const uint32_t bucket = sh.bucket;
      __syncthreads();
      if (bucket == rem) break;
      hb = lb - 1;
    }
  }
  // keys below the boundary bucket fill [0, k - rem), boundary keys fill
  // [k - rem, k) until rem are taken (take_all: every key)
  const uint64_t hi_key = take_all ? ~0ull : (prefix | ~pmask);
  const uint64_t lt_key = take_all ? 0ull : prefix;
  const uint32_t nlt = take_all ? 0u : (uint32_t)k - rem;
  uint32_t clt = 0, ceq = 0;
#pragma unroll
  for (int u = 0; u < KPT; ++u)
    if (valid(u)) {
      clt += v[u] < lt_key ? 1u : 0u;
      ceq += (v[u] >= lt_key && v[u] <= hi_key) ? 1u : 0u;
    }
  uint32_t tot;
  const uint32_t ex = block_excl_scan<NT>((clt << 16) | ceq, sh.wsum, &tot);
  uint32_t plt = ex >> 16, peq = ex & 0xFFFFu;
  uint64_t mx = 0;
#pragma unroll
  for (int u = 0; u < KPT; ++u)
    if (valid(u)) {
      if (v[u] < lt_key) {
        dst[plt++] = v[u];
        mx = v[u] > mx ? v[u] : mx;
      } else if (v[u] <= hi_key) {
        if (peq < rem) {
          dst[nlt + peq] = v[u];
          mx = v[u] > mx ? v[u] : mx;
        }
        ++peq;
      }
    }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if (lane == 0) sh.hi[wave] = mx;
  __syncthreads();
  uint64_t kth = sh.hi[0];
#pragma unroll
  for (int w = 1; w < NW; ++w) kth = sh.hi[w] > kth ? sh.hi[w] : kth;
  __syncthreads();
  return take_all ? KEY_NONE : kth;
}

// ---------------------------------------------------------------------------
// Code scan (query-major popcount form). One workgroup per (query, probe)
// item, ordered probe-rank-major so that every query's nearest lists are
// scanned first. Each lane takes one vector of a 64-vector micro-block:
//   ip  = sum_t 2^t popcount(code & plane_t)      (exact integer)
//   pop = popcount(code)
//   E   = v_l (2 pop - D) + Delta (2 ip - sum qu)  (= sum_d b_d (v_l + Delta qu_d))
//   d_hat^2 = ||r||^2 + n_x^2 - 2 n_x E / (sqrt(D) alpha_x)
// with the two per-vector factors stored folded (n_x^2, -2 n_x/(sqrt(D) alpha)).
// Candidates below the running threshold go to an LDS buffer that is cut back
// to the best R whenever it could overflow; the item's final R-th estimate
// tightens the query's global bound (the IVF-aware pruning of Sec. 3.3.3).
// ---------------------------------------------------------------------------

__device__ void sel_compact(uint64_t* sel, int cap, int R, int* s_n, uint64_t* s_thr) {
  const int n = *s_n;
  for (int t = n + threadIdx.x; t < cap; t += blockDim.x) sel[t] = KEY_NONE;
  __syncthreads();
  bitonic_sort_lds(sel, cap);
  if (threadIdx.x == 0 && n >= R) {
    *s_thr = sel[R - 1];
    *s_n = R;
  }
  __syncthreads();
}

// LDS of the popcount scan's radix cut-back.
struct PopcCutShared {
  uint32_t hist[256];
  uint32_t wsum[4];
  uint32_t digit, rem, bucket, nlt, neq;
  uint64_t lo[4], hi[4];
};

// The k smallest of the unique keys src[0..n) (k < n) written to dst[0..k)
// in any order by a 256-thread workgroup; returns the k-th smallest. An
// MSB-first radix select whose passes read the keys from LDS (8-bit digits
// from the highest bit in which the keys differ), so the caller's registers
// stay free; keys below the boundary digit and the boundary bucket (taken
// whole) are then appended with one LDS atomic per wave. src and dst must not
// overlap. Ends with a barrier.
__device__ uint64_t popc_radix_cut(const uint64_t* src, int n, int k, uint64_t* dst, PopcCutShared& sh) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t lo = ~0ull, hi = 0;
  for (int t = tid; t < n; t += 256) {
    const uint64_t x = src[t];
    lo = x < lo ? x : lo;
    hi = x > hi ? x : hi;
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t l2 = __shfl_xor(lo, off), h2 = __shfl_xor(hi, off);
    lo = l2 < lo ? l2 : lo;
    hi = h2 > hi ? h2 : hi;
  }
  if (lane == 0) {
    sh.lo[wave] = lo;
    sh.hi[wave] = hi;
  }
  if (tid == 0) sh.nlt = sh.neq = 0u;
  __syncthreads();
  lo = sh.lo[0];
  hi = sh.hi[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) {
    lo = sh.lo[w] < lo ? sh.lo[w] : lo;
    hi = sh.hi[w] > hi ? sh.hi[w] : hi;
  }
  const uint64_t diff = lo ^ hi;
  const int top = diff ? 63 - __clzll((long long)diff) : -1;
  uint64_t prefix = 0, pmask = 0;
  if (top < 63) {
    pmask = top < 0 ? ~0ull : ~((2ull << top) - 1ull);
    prefix = lo & pmask;
  }
  uint32_t rem = (uint32_t)k;
  for (int hb = top; hb >= 0;) {
    const int lb = hb >= 7 ? hb - 7 : 0;
    const uint64_t dmask = (2ull << (hb - lb)) - 1ull;
    sh.hist[tid] = 0u;
    __syncthreads();
    for (int t = tid; t < n; t += 256) {
      const uint64_t x = src[t];
      if ((x & pmask) == prefix) atomicAdd(&sh.hist[(x >> lb) & dmask], 1u);
    }
    __syncthreads();
    const uint32_t h = sh.hist[tid];
    const uint32_t incl = hist_incl_scan<256>(h, sh.wsum);
    const uint32_t excl = incl - h;
    if (excl < rem && rem <= incl) {
      sh.digit = (uint32_t)tid;
      sh.rem = rem - excl;
      sh.bucket = h;
    }
    __syncthreads();
    prefix |= (uint64_t)sh.digit << lb;
    pmask |= dmask << lb;
    rem = sh.rem;
    const uint32_t bucket = sh.bucket;
    __syncthreads();
    if (bucket == rem) break;
    hb = lb - 1;
  }
  // keys below the prefix fill [0, k - rem), boundary keys [k - rem, k)
  const uint64_t hi_key = prefix | ~pmask;
  const uint32_t nlt = (uint32_t)k - rem;
  uint64_t mx = 0;
  for (int t0 = 0; t0 < n; t0 += 256) {
    const int t = t0 + tid;
    const uint64_t x = t < n ? src[t] : KEY_NONE;
    const bool blt = t < n && x < prefix;
    const bool beq = t < n && x >= prefix && x <= hi_key;
    const uint64_t mlt = __ballot(blt), meq = __ballot(beq);
    uint32_t b0 = 0, e0 = 0;
    if (lane == 0) {
      if (mlt) b0 = atomicAdd(&sh.nlt, (uint32_t)__popcll(mlt));
      if (meq) e0 = atomicAdd(&sh.neq, (uint32_t)__popcll(meq));
    }
    b0 = (uint32_t)__shfl(b0, 0);
    e0 = (uint32_t)__shfl(e0, 0);
    if (blt) {
      dst[b0 + lane_prefix(mlt)] = x;
      mx = x > mx ? x : mx;
    }
    if (beq) {
      const uint32_t q = e0 + lane_prefix(meq);
      if (q < rem) {
        dst[nlt + q] = x;
        mx = x > mx ? x : mx;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if (lane == 0) sh.hi[wave] = mx;
  __syncthreads();
  uint64_t kth = sh.hi[0];
#pragma unroll
  for (int w = 1; w < 4; ++w) kth = sh.hi[w] > kth ? sh.hi[w] : kth;
  __syncthreads();
  return kth;
}

// Buffers of up to this many keys are cut back by popc_radix_cut into a
// second buffer of the same size, in the instances with a fixed word count of
// at most 8 (D <= 256); longer buffers and the wide instances use an LDS
// bitonic sort in place.
constexpr int kPopcRadixCap = 1024;
template <int WT>
__host__ __device__ constexpr bool popc_radix_form() { return WT > 0 && WT <= 8; }

template <int WT, int BQT, bool DUMP>
__global__ __launch_bounds__(256) void k_scan_popc(ScanArgs a, int cap) {
  extern __shared__ uint64_t sel[];  // cap keys (two buffers of cap in the radix form)
  __shared__ uint32_t s_cnt[3];  // appends of round r counted in s_cnt[r % 3]
  __shared__ PopcCutShared cs;
  const bool radix = popc_radix_form<WT>() && cap <= kPopcRadixCap;
  uint64_t* buf = sel;          // the buffer being filled
  uint64_t* spare = sel + cap;  // (radix) the other one
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int W = WT > 0 ? WT : a.L.W;
  const int BQ = BQT > 0 ? BQT : a.Q.bqs;
  const int bqs = a.Q.bqs;
  const int it = blockIdx.x;
  const int pr = it / a.nq, i = it - pr * a.nq;
  const int p = a.p0 + pr;
  if (a.qmask && a.qmask[i] == 0u) return;  // uniform over the workgroup
  const int64_t pair = (int64_t)i * a.nprobe + p;
  const int j = a.probes[pair];
  const int len = j >= 0 ? a.L.list_len[j] : 0, mb0 = j >= 0 ? a.L.list_mb[j] : 0;
  const int nmb = (len + 63) >> 6;
  const int R = a.R;
  const uint32_t* planes = a.Q.planes + pair * W * bqs;
  const float4 sc = a.Q.scal[pair];
  const float rn2 = sc.x, vl = sc.y, delta = sc.z;
  const int sumqu = (int)sc.w;
  const int D = a.L.d;
  if (tid == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = 0u;
  // the threshold key (the same in every thread; lowered by each compaction)
  uint64_t thr = a.qthr ? ((static_cast<uint64_t>(a.qthr[i]) << 32) | 0xFFFFFFFFull) : KEY_NONE;
  const size_t rec = (size_t)(W + 2) * 64;
  // For the fixed word counts a micro-block's words (codes, then the two
  // factor rows) are loaded into registers one round ahead, so the next
  // block's loads are in flight while this one is computed.
  constexpr bool PF = WT > 0 && WT <= 8;
  constexpr int NR = PF ? WT + 2 : 1;
  uint32_t nx[NR];
  auto fetch = [&](int m) __attribute__((always_inline)) {
    const uint32_t* blk = a.L.blocks + (size_t)(mb0 + m) * rec;
#pragma unroll
    for (int w = 0; w < NR; ++w) nx[w] = blk[w * 64 + lane];
  };
  if (PF && wave < nmb) fetch(wave);
  __syncthreads();  // s_cnt cleared
  // buffer fill (the same value in every thread) and round number: round r
  // appends behind the fill through s_cnt[r % 3]; the counter of round r + 1
  // is cleared during round r (its last readers, after round r - 2's
  // barrier, are all past round r - 1's), so one barrier per round gives
  // every thread the same fill
  int fill = 0, rr = 0;
  for (int base = 0; base < nmb; base += 4) {
    const int m = base + wave;
    const int par = rr % 3;
    if (tid == 0) s_cnt[(rr + 1) % 3] = 0u;
    uint64_t key = KEY_NONE;
    if (m < nmb) {
      const uint32_t* blk = a.L.blocks + (size_t)(mb0 + m) * rec;
      uint32_t cur[NR];
      if constexpr (PF) {
#pragma unroll
        for (int w = 0; w < NR; ++w) cur[w] = nx[w];
        if (m + 4 < nmb) fetch(m + 4);
      }
      // (bit-plane counts in registers: the plane loops run over the
      // instance's plane count, or all 8 with a guard)
      constexpr int NBQ = BQT > 0 ? BQT : 8;
      int acc[NBQ];
#pragma unroll
      for (int t = 0; t < NBQ; ++t) acc[t] = 0;
      int pop = 0;
      auto word = [&](int w) __attribute__((always_inline)) {
        const uint32_t c = PF ? cur[w] : blk[w * 64 + lane];
        pop += __popc(c);
#pragma unroll
        for (int t = 0; t < NBQ; ++t)
          if (t < BQ) acc[t] += __popc(c & planes[w * bqs + t]);
      };
      if constexpr (WT > 0) {
#pragma unroll
        for (int w = 0; w < WT; ++w) word(w);
      } else {
        for (int w = 0; w < W; ++w) word(w);
      }
      int ip = 0;
#pragma unroll
      for (int t = 0; t < NBQ; ++t) ip += t < BQ ? acc[t] << t : 0;
      const float fadd = __uint_as_float(PF ? cur[NR - 2] : blk[W * 64 + lane]);
      const float fmul = __uint_as_float(PF ? cur[NR - 1] : blk[(W + 1) * 64 + lane]);
      const float est = rbq_estimate(rn2, vl, delta, -sumqu, ip, fadd, fmul, rbq_vx(fmul, pop, D));
      const int v = (m << 6) + lane;
      if (v < len) {
        key = key64(est, (uint32_t)((mb0 << 6) + v));
        if (DUMP) {
          a.dump_ip[pair * a.maxlen + v] = ip;
          a.dump_est[pair * a.maxlen + v] = est;
        }
      }
    }
    const bool pass = key < thr;
    const uint64_t mask = __ballot(pass);
    if (mask) {
      uint32_t off = 0;
      if (lane == 0) off = (uint32_t)fill + atomicAdd(&s_cnt[par], (uint32_t)__popcll(mask));
      off = __shfl(off, 0);
      if (pass) buf[off + lane_prefix(mask)] = key;
    }
    __syncthreads();
    fill += (int)s_cnt[par];
    ++rr;
    if (fill > cap - 256) {  // the next round could overflow: keep the best R
      if (radix) {  // (fill > cap - 256 >= R)
        thr = popc_radix_cut(buf, fill, R, spare, cs);
        uint64_t* t = buf;
        buf = spare;
        spare = t;
        fill = R;
      } else {
        for (int t = fill + tid; t < cap; t += 256) buf[t] = KEY_NONE;
        __syncthreads();
        bitonic_sort_lds(buf, cap);  // (ends with a barrier)
        if (fill >= R) {
          thr = buf[R - 1];
          fill = R;
        }
      }
    }
  }
  const int n = fill;
  // keep the best R (an item with at most R survivors keeps them all, unsorted)
  uint64_t rth = KEY_NONE;  // the R-th smallest key when n > R
  if (n > R && radix) {
    rth = popc_radix_cut(buf, n, R, spare, cs);
    buf = spare;
  } else if (n > R) {
    int P = 2;
    while (P < n) P <<= 1;
    for (int t = n + tid; t < P; t += 256) buf[t] = KEY_NONE;
    __syncthreads();
    bitonic_sort_lds(buf, P);
    rth = buf[R - 1];
  }
  // append this item's survivors (at most R) to the query's pool; the pool
  // holds R * (probe ranks in this launch) keys, so it cannot overflow
  const int nout = n < R ? n : R;
  __shared__ int s_base;
  if (tid == 0) s_base = nout ? (int)atomicAdd(&a.pcnt[i], (uint32_t)nout) : 0;
  __syncthreads();
  uint64_t* dst = a.out + (int64_t)i * a.out_ld + R + s_base;
  for (int r = tid; r < nout; r += 256) {
    const uint64_t sv = buf[r];
    const int id = a.L.pos2id[(uint32_t)sv];
    dst[r] = (sv & 0xFFFFFFFF00000000ull) | (uint32_t)id;
  }
  if (a.qthr && tid == 0 && n > R) atomicMin(&a.qthr[i], (uint32_t)(rth >> 32));
}

template <int WT, int BQT>
static void scan_dispatch(hipStream_t s, const ScanArgs& a, int cap, bool dump) {
  const unsigned items = (unsigned)((int64_t)a.nq * a.pn);
  const size_t lds = (size_t)(popc_radix_form<WT>() && cap <= kPopcRadixCap ? 2 : 1) * cap * sizeof(uint64_t);
  if (dump)
    hipLaunchKernelGGL((k_scan_popc<WT, BQT, true>), dim3(items), dim3(256), lds, s, a, cap);
  else
    hipLaunchKernelGGL((k_scan_popc<WT, BQT, false>), dim3(items), dim3(256), lds, s, a, cap);
}

void launch_scan_popc(hipStream_t s, const ScanArgs& a) {
  if ((int64_t)a.nq * a.pn <= 0) return;
  const int cap = pow2_at_least(a.R + 256);
  const bool dump = a.dump_ip != nullptr;
  const int bq4 = a.Q.bqs == 4;
  if (bq4 && a.L.W == 4)
    scan_dispatch<4, 4>(s, a, cap, dump);
  else if (bq4 && a.L.W == 3)
    scan_dispatch<3, 4>(s, a, cap, dump);
  else if (bq4 && a.L.W == 30)
    scan_dispatch<30, 4>(s, a, cap, dump);
  else
    scan_dispatch<0, 0>(s, a, cap, dump);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Query-major scan with the unquantised residual. The item's residual
// r = P^T q - P^T c_j is formed in LDS (zero past d), its squared norm summed
// in a fixed order, and a table lut[g][m] = sum_i s_i r_{GB g + i}, s_i = +1
// for bit i of m set and -1 otherwise, is built for every group g of GB
// dimensions. A vector's E = sum_d b_d r_d is then one lookup per group of its
// code, summed in group order; the rest (threshold, LDS selection, pools) is
// the popcount scan's.
// ---------------------------------------------------------------------------
constexpr int kLutMaxD = 1024;

template <int GB, bool DUMP>
__global__ __launch_bounds__(256) void k_scan_lut(ScanArgs a, int cap) {
  extern __shared__ uint64_t sel[];
  constexpr int NE = 1 << GB;                    // table entries per group
  constexpr int NG = (GB == 8 ? 128 : kLutMaxD) / GB;  // groups held (16 KB of table)
  __shared__ float lut[NG * NE];
  __shared__ float rs[NG * GB];
  __shared__ float red[256];
  __shared__ int s_n;
  __shared__ uint64_t s_thr;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int W = a.L.W;
  const int D = a.L.d;
  const int ng = (D + GB - 1) / GB;
  const int it = blockIdx.x;
  const int pr = it / a.nq, i = it - pr * a.nq;
  const int p = a.p0 + pr;
  if (a.qmask && a.qmask[i] == 0u) return;  // uniform over the workgroup
  const int64_t pair = (int64_t)i * a.nprobe + p;
  const int j = a.probes[pair];
  const int len = j >= 0 ? a.L.list_len[j] : 0, mb0 = j >= 0 ? a.L.list_mb[j] : 0;
  const int nmb = (len + 63) >> 6;
  const int R = a.R;
  if (len == 0) return;  // nothing to scan (uniform)
  // the residual and its squared norm (each thread sums a fixed stride)
  float part = 0.f;
  for (int d = tid; d < ng * GB; d += 256) {
    const float r = d < D ? a.qrot[(int64_t)i * a.ldq + d] - a.crot[(int64_t)j * a.ldc + d] : 0.f;
    rs[d] = r;
    part = fmaf(r, r, part);
  }
  red[tid] = part;
  if (tid == 0) {
    s_n = 0;
    s_thr = a.qthr ? ((static_cast<uint64_t>(a.qthr[i]) << 32) | 0xFFFFFFFFull) : KEY_NONE;
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (tid < off) red[tid] += red[tid + off];
    __syncthreads();
  }
  const float rn2 = red[0];
  // the sign-pattern tables, each entry summed in dimension order
  for (int e = tid; e < ng * NE; e += 256) {
    const int g = e / NE, m = e - g * NE;
    float acc = 0.f;
#pragma unroll
    for (int b = 0; b < GB; ++b) {
      const float r = rs[g * GB + b];
      acc += ((m >> b) & 1) ? r : -r;
    }
    lut[e] = acc;
  }
  __syncthreads();
  const size_t rec = (size_t)(W + 2) * 64;
  for (int base = 0; base < nmb; base += 4) {
    const int m = base + wave;
    uint64_t key = KEY_NONE;
    if (m < nmb) {
      const uint32_t* blk = a.L.blocks + (size_t)(mb0 + m) * rec;
      float E = 0.f;
      for (int w = 0; w < W; ++w) {
        const uint32_t c = blk[w * 64 + lane];
#pragma unroll
        for (int t = 0; t < 32 / GB; ++t) {
          const int g = w * (32 / GB) + t;
          if (g < ng) E += lut[g * NE + ((c >> (GB * t)) & (NE - 1))];
        }
      }
      const float fadd = __uint_as_float(blk[W * 64 + lane]);
      const float fmul = __uint_as_float(blk[(W + 1) * 64 + lane]);
      const float est = fmaf(fmul, E, fadd) + rn2;
      const int v = (m << 6) + lane;
      if (v < len) {
        key = key64(est, (uint32_t)((mb0 << 6) + v));
        if (DUMP) a.dump_est[pair * a.maxlen + v] = est;
      }
    }
    const uint64_t thr = s_thr;
    const bool pass = key < thr;
    const uint64_t mask = __ballot(pass);
    if (mask) {
      int off = 0;
      if (lane == 0) off = atomicAdd(&s_n, (int)__popcll(mask));
      off = __shfl(off, 0);
      if (pass) sel[off + (int)lane_prefix(mask)] = key;
    }
    __syncthreads();
    const int nn = s_n;
    __syncthreads();  // every thread has read the count before the next appends
    if (nn > cap - 256) sel_compact(sel, cap, R, &s_n, &s_thr);
  }
  __syncthreads();
  const int n = s_n;
  if (n > R) {  // keep the best R
    int P = 2;
    while (P < n) P <<= 1;
    for (int t = n + tid; t < P; t += 256) sel[t] = KEY_NONE;
    __syncthreads();
    bitonic_sort_lds(sel, P);
  }
  const int nout = n < R ? n : R;
  __shared__ int s_base;
  if (tid == 0) s_base = nout ? (int)atomicAdd(&a.pcnt[i], (uint32_t)nout) : 0;
  __syncthreads();
  uint64_t* dst = a.out + (int64_t)i * a.out_ld + R + s_base;
  for (int r = tid; r < nout; r += 256) {
    const uint64_t sv = sel[r];
    const int id = a.L.pos2id[(uint32_t)sv];
    dst[r] = (sv & 0xFFFFFFFF00000000ull) | (uint32_t)id;
  }
  if (a.qthr && tid == 0 && n > R) atomicMin(&a.qthr[i], (uint32_t)(sel[R - 1] >> 32));
}

int scan_lut_max_d() { return kLutMaxD; }

void launch_scan_lut(hipStream_t s, const ScanArgs& a) {
  if ((int64_t)a.nq * a.pn <= 0) return;
  RBQ_CHECK(a.L.d <= kLutMaxD, "the unquantised-query scan supports d <= 1024");
  RBQ_CHECK(a.qrot && a.crot, "unquantised-query scan: rotated queries and centroids");
  const int cap = pow2_at_least(a.R + 256);
  const unsigned items = (unsigned)((int64_t)a.nq * a.pn);
  const size_t lds = (size_t)cap * sizeof(uint64_t);
  const bool dump = a.dump_est != nullptr;
  if (a.L.d <= 128) {
    if (dump)
      hipLaunchKernelGGL((k_scan_lut<8, true>), dim3(items), dim3(256), lds, s, a, cap);
    else
      hipLaunchKernelGGL((k_scan_lut<8, false>), dim3(items), dim3(256), lds, s, a, cap);
  } else {
    if (dump)
      hipLaunchKernelGGL((k_scan_lut<4, true>), dim3(items), dim3(256), lds, s, a, cap);
    else
      hipLaunchKernelGGL((k_scan_lut<4, false>), dim3(items), dim3(256), lds, s, a, cap);
  }
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Fused query-major scan + selection for chunks whose lists are shared by few
// queries: one workgroup (8 waves, 64 KB of LDS: two per CU) per query loads
// the query's running top-R into an LDS buffer, scans the chunk's probed lists
// (popcount inner products, the same estimator expression as the other
// scans), appends every estimate at or below the query's threshold, and
// whenever the buffer could overflow keeps only its best R and lowers the
// threshold to their R-th estimate. The selection holds the buffer in
// registers (an MSB-first radix select with fire-and-forget histogram atomics,
// positions from one workgroup scan). Each wave takes every eighth micro-block
// of the chunk's lists with the data of its next two loaded ahead (two register
// sets, alternate rounds). At the end the best R become the query's running
// top-R and its threshold. Nothing goes through the global pool.
// ---------------------------------------------------------------------------

constexpr int kFusedNT = 512;                 // threads per workgroup
constexpr int kFusedKPT = 16;                 // buffer keys per thread in a selection
constexpr int kFusedCap = kFusedNT * kFusedKPT;  // LDS buffer keys (64 KB)

// Sorted top-k of a row of float scores (key = ordered score << 32 | column):
// the row in registers (16 per thread), the k smallest selected, then an LDS
// bitonic sort of those k.
template <int NT, int KPT>
__global__ __launch_bounds__(NT) void k_score_topk(TopkArgs a) {
  extern __shared__ uint64_t sel[];  // KP keys
  __shared__ SelRegShared<NT> sh;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const int k = a.rowk ? a.rowk[row] : a.k;
  const int n = a.ncols;
  uint64_t v[KPT];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int c = u * NT + tid;
    v[u] = c < n ? key64(a.score[row * a.ld + c], (uint32_t)c) : KEY_NONE;
  }
  (void)select_regs<NT, KPT>(v, n, k, sel, sh);
  for (int t = min(n, k) + tid; t < a.KP; t += NT) sel[t] = KEY_NONE;
  __syncthreads();
  bitonic_sort_lds(sel, a.KP);
  for (int t = tid; t < k; t += NT) {
    const uint64_t x = sel[t];
    if (a.out_keys) a.out_keys[row * a.ldo + t] = x;
    if (a.out_low) a.out_low[row * k + t] = x == KEY_NONE ? -1 : (int32_t)(uint32_t)x;
    if (a.out_val) a.out_val[row * k + t] = x == KEY_NONE ? INFINITY : f32_ord((uint32_t)(x >> 32));
  }
}

// Appends the keys whose pass flag is set to kept[] at the running count
// *cnt (LDS): one ballot per key slot and one LDS atomic per wave.
template <int U>
__device__ inline void append_kept(const uint64_t (&key)[U], const bool (&pass)[U], uint64_t* kept,
                                   uint32_t* cnt) {
  const int lane = threadIdx.x & 63;
  uint64_t bal[U];
  uint32_t wtot = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    bal[u] = __ballot(pass[u]);
    wtot += (uint32_t)__popcll(bal[u]);
  }
  if (wtot == 0) return;  // (uniform per wave)
  uint32_t base = 0;
  if (lane == 0) base = atomicAdd(cnt, wtot);
  base = (uint32_t)__shfl(base, 0);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (pass[u])
      kept[base + (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal[u] >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bal[u], 0u))] = key[u];
    base += (uint32_t)__popcll(bal[u]);
  }
}

// Sorted top-k of a score row longer than one register-resident piece, one
// workgroup per row. A bound comes from the first NT x KPT scores: for
// k <= NT / 2 the k-th smallest of the threads' minima (k distinct keys lie
// at or below it), else the k-th smallest of all of them. The first piece's
// keys up to the bound are kept (in LDS); the rest of the row streams past in
// tiles of NT x U scores and only keys below the bound are kept. A key above
// the bound has k smaller keys before it, so the kept keys hold the row's k
// smallest. When the next tile might not fit, the kept keys are cut back to
// their k smallest and the bound drops to the new k-th key. LDS: NT x KPT keys
// (dynamic), which must leave room for k keys plus one tile.
template <int NT, int KPT, int U, int PD, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void k_score_topk_long(TopkArgs a) {
  constexpr int CAP = NT * KPT, TILE = NT * U;
  extern __shared__ uint64_t kept[];  // CAP keys
  __shared__ SelRegShared<NT> sh;
  __shared__ uint32_t s_cnt;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const float* src = a.score + row * a.ld;
  const int n = a.ncols, k = a.k;  // n > CAP and k <= CAP - TILE (launcher)
  uint64_t v[KPT];
#pragma unroll
  for (int u = 0; u < KPT; ++u) {
    const int c = u * NT + tid;
    v[u] = key64(src[c], (uint32_t)c);
  }
  // the scores of the next PD tiles are loaded ahead, so their loads are in
  // flight during the selection, the appends and the barriers before them
  float f[PD][U];
  auto load_tile = [&](int c0, float (&dst)[U]) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * NT + tid;
      dst[u] = c < n ? src[c] : 0.f;
    }
  };
#pragma unroll
  for (int p = 0; p < PD; ++p) load_tile(CAP + p * TILE, f[p]);
  uint64_t bound;
  uint32_t cnt;
  if (k <= NT / 2) {
    uint64_t m[1] = {v[0]};
#pragma unroll
    for (int u = 1; u < KPT; ++u) m[0] = v[u] < m[0] ? v[u] : m[0];
    bound = select_regs<NT, 1>(m, NT, k, kept, sh);  // (kept[] as scratch; ends with a barrier)
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    bool pass[KPT];
#pragma unroll
    for (int u = 0; u < KPT; ++u) pass[u] = v[u] <= bound;
    append_kept<KPT>(v, pass, kept, &s_cnt);
    __syncthreads();
    cnt = s_cnt;
  } else {
    bound = select_regs<NT, KPT>(v, CAP, k, kept, sh);
    cnt = (uint32_t)k;
    if (tid == 0) s_cnt = cnt;
  }
  __syncthreads();  // (every thread has the count before the next change to it)
  for (int c0 = CAP; c0 < n; c0 += TILE) {
    if (cnt > (uint32_t)(CAP - TILE)) {  // (uniform) cut back to the k smallest
#pragma unroll
      for (int u = 0; u < KPT; ++u) {
        const int i = u * NT + tid;
        v[u] = i < (int)cnt ? kept[i] : KEY_NONE;
      }
      bound = select_regs<NT, KPT>(v, (int)cnt, k, kept, sh);
      cnt = (uint32_t)k;
      if (tid == 0) s_cnt = cnt;
      __syncthreads();
    }
    float fn[U];
    load_tile(c0 + PD * TILE, fn);
    uint64_t key[U];
    bool pass[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = c0 + u * NT + tid;
      key[u] = key64(f[0][u], (uint32_t)c);
      pass[u] = c < n && key[u] < bound;
    }
#pragma unroll
    for (int p = 0; p + 1 < PD; ++p)
#pragma unroll
      for (int u = 0; u < U; ++u) f[p][u] = f[p + 1][u];
#pragma unroll
    for (int u = 0; u < U; ++u) f[PD - 1][u] = fn[u];
    append_kept<U>(key, pass, kept, &s_cnt);
    __syncthreads();
    cnt = s_cnt;
    __syncthreads();  // (every thread has read the count before the next tile adds to it)
  }
  if (cnt > (uint32_t)k) {
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
      const int i = u * NT + tid;
      v[u] = i < (int)cnt ? kept[i] : KEY_NONE;
    }
    (void)select_regs<NT, KPT>(v, (int)cnt, k, kept, sh);
  }
  for (int t = k + tid; t < a.KP; t += NT) kept[t] = KEY_NONE;
  __syncthreads();
  bitonic_sort_lds(kept, a.KP);
  for (int t = tid; t < k; t += NT) {
    const uint64_t x = kept[t];
    if (a.out_keys) a.out_keys[row * a.ldo + t] = x;
    if (a.out_low) a.out_low[row * k + t] = x == KEY_NONE ? -1 : (int32_t)(uint32_t)x;
    if (a.out_val) a.out_val[row * k + t] = x == KEY_NONE ? INFINITY : f32_ord((uint32_t)(x >> 32));
  }
}

// Two shapes: up to 4096 selected keys from a first piece of 8192 scores
// (512 threads, 64 KB of LDS, two rows per CU, one tile of 4096 loaded
// ahead), and for k <= 256 a first piece of 2048 scores (256 threads, 16 KB,
// five rows per CU, two tiles of 1024 ahead), so that more score bytes are in
// flight per CU.
template <int NT, int KPT, int U, int PD, int WPE>
static void launch_score_topk_long_as(hipStream_t s, const TopkArgs& a, int rows) {
  constexpr int cap = NT * KPT;
  RBQ_CHECK(a.ncols > cap && a.k <= cap - NT * U && a.KP <= cap, "long score top-k: shape");
  const size_t lds = (size_t)cap * sizeof(uint64_t);
  auto kern = k_score_topk_long<NT, KPT, U, PD, WPE>;
  static std::once_flag attr_once;
  std::call_once(attr_once, [&] {
    RBQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  });
  hipLaunchKernelGGL(kern, dim3((unsigned)rows), dim3(NT), lds, s, a);
  RBQ_HIP(hipGetLastError());
}

static void launch_score_topk_long(hipStream_t s, const TopkArgs& a, int rows) {
  if (a.k <= 256)
    launch_score_topk_long_as<256, 8, 4, 2, 5>(s, a, rows);
  else
    launch_score_topk_long_as<512, 16, 8, 1, 4>(s, a, rows);
}

static void launch_score_topk(hipStream_t s, const TopkArgs& a, int rows) {
  RBQ_CHECK(a.ncols <= kScoreTopkCols && a.KP >= a.k, "score top-k: row too long");
  if (a.ncols <= 256 * 16)
    hipLaunchKernelGGL((k_score_topk<256, 16>), dim3(rows), dim3(256), (size_t)a.KP * sizeof(uint64_t), s, a);
  else
    hipLaunchKernelGGL((k_score_topk<512, 16>), dim3(rows), dim3(512), (size_t)a.KP * sizeof(uint64_t), s, a);
  RBQ_HIP(hipGetLastError());
}

// One micro-block's data for the fused scan, loaded ahead: per lane its
// vector's code words, factors and id; per wave (uniform, scalar loads) the
// pair's bit-planes and scalars and the block's place in its list.
template <int WR, int PR>
struct FusedSlot {
  uint32_t cw[WR];
  float fa, fm;
  int id;
  uint32_t pl[PR];
  float4 sc;
  int len, mb;
  int64_t pair;
};

__device__ inline int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }

template <int WT, int BQT>
__global__ __launch_bounds__(kFusedNT) void k_scan_fused(FusedArgs a) {
  constexpr int NT = kFusedNT, NW = NT / 64, KPT = kFusedKPT;
  constexpr int WR = WT > 0 ? WT : 32;
  constexpr int PR = (WT > 0 && BQT > 0) ? WT * BQT : 1;  // bit-plane words kept ahead
  extern __shared__ uint64_t buf[];  // a.cap keys
  __shared__ SelRegShared<NT> sh;
  __shared__ int32_t s_pre[257];
  __shared__ int32_t s_lpos[256], s_llen[256];  // the group's lists: first position, length
  __shared__ uint32_t s_n, s_thr;
  __shared__ uint32_t s_cnt[3];  // appends of round r counted in s_cnt[r % 3]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = uniform_i32(tid >> 6);
  const int i = blockIdx.x;
  if (a.qmask && a.qmask[i] == 0u) return;  // uniform over the workgroup
  const int W = WT > 0 ? WT : a.L.W;
  const int BQ = BQT > 0 ? BQT : a.Q.bqs;
  const int bqs = a.Q.bqs;
  const int D = a.L.d;
  const int Rq = a.rowk ? a.rowk[i] : a.R;
  uint64_t* row = a.out + (int64_t)i * a.out_ld;
  const size_t rec = (size_t)(W + 2) * 64;
  if (tid == 0) {
    s_n = 0;
    s_thr = a.reset ? 0xFFFFFFFFu : a.qthr[i];
    s_cnt[0] = s_cnt[1] = s_cnt[2] = 0u;
  }
  __syncthreads();
  // the running top-R (none when starting afresh)
  for (int r0 = 0; r0 < (a.reset ? 0 : a.R); r0 += NT) {
    const int r = r0 + tid;
    const uint64_t key = r < a.R ? row[r] : KEY_NONE;
    const bool t = key != KEY_NONE;
    const uint64_t m = __ballot(t);
    uint32_t base = 0;
    if (lane == 0 && m) base = atomicAdd(&s_n, (uint32_t)__popcll(m));
    base = __shfl(base, 0);
    if (t) buf[base + lane_prefix(m)] = key;
  }
  __syncthreads();
  // buffer fill (the same value in every thread) and round number
  int fill = (int)s_n;
  int rr = 0;
  // keep the best Rq of the buffer and lower the threshold (whole workgroup)
  auto shrink = [&]() __attribute__((always_inline)) {
    const int n = fill;
    uint64_t v[KPT];
#pragma unroll
    for (int u = 0; u < KPT; ++u) {
      const int c = u * NT + tid;
      v[u] = c < n ? buf[c] : KEY_NONE;
    }
    __syncthreads();  // every key read before any is overwritten
    const uint64_t kth = select_regs<NT, KPT>(v, n, Rq, buf, sh);
    fill = min(n, Rq);
    if (tid == 0) {
      if (kth != KEY_NONE) {
        const uint32_t t = (uint32_t)(kth >> 32);
        if (t < s_thr) s_thr = t;
      }
    }
    __syncthreads();
  };
  for (int s0 = 0; s0 < a.pn; s0 += 256) {
    const int sn = min(256, a.pn - s0);
    int cntmb = 0;
    if (tid < sn) {
      const int j = a.probes[(int64_t)i * a.nprobe + a.p0 + s0 + tid];
      const int len = j >= 0 ? a.L.list_len[j] : 0;
      cntmb = (len + 63) >> 6;
      s_llen[tid] = len;
      s_lpos[tid] = j >= 0 ? a.L.list_mb[j] << 6 : 0;
    }
    const uint32_t incl = hist_incl_scan<NT>((uint32_t)cntmb, sh.wsum);
    if (tid < sn) s_pre[tid + 1] = (int32_t)incl;
    if (tid == 0) s_pre[0] = 0;
    __syncthreads();
    const int total = uniform_i32(s_pre[sn]);
    auto load = [&](int idx, FusedSlot<WR, PR>& f) __attribute__((always_inline)) {  // idx: wave-uniform
      int lo = 0, hi = sn;  // s_pre[lo] <= idx < s_pre[hi]
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (uniform_i32(s_pre[mid]) <= idx)
          lo = mid;
        else
          hi = mid;
      }
      f.mb = idx - uniform_i32(s_pre[lo]);
      f.pair = (int64_t)i * a.nprobe + a.p0 + s0 + lo;
      f.len = uniform_i32(s_llen[lo]);
      const int pos0 = uniform_i32(s_lpos[lo]);
      const uint32_t* blk = a.L.blocks + (size_t)((pos0 >> 6) + f.mb) * rec;
#pragma unroll
      for (int w = 0; w < WR; ++w)
        if (w < W) f.cw[w] = blk[w * 64 + lane];
      f.fa = __uint_as_float(blk[W * 64 + lane]);
      f.fm = __uint_as_float(blk[(W + 1) * 64 + lane]);
      const int v = (f.mb << 6) + lane;
      f.id = v < f.len ? a.L.pos2id[pos0 + v] : 0;
      f.sc = a.Q.scal[f.pair];
      if (PR > 1) {
        const uint32_t* planes = a.Q.planes + f.pair * W * bqs;
#pragma unroll
        for (int w = 0; w < (WT > 0 ? WT : 1); ++w)
#pragma unroll
          for (int t = 0; t < (BQT > 0 ? BQT : 1); ++t) f.pl[(w * (BQT > 0 ? BQT : 1) + t) % PR] = planes[w * bqs + t];
      }
    };
    // estimates of one micro-block; survivors appended to the buffer
    auto scan = [&](const FusedSlot<WR, PR>& f, int par) __attribute__((always_inline)) {
      const uint32_t* planes = a.Q.planes + f.pair * W * bqs;
      int acc[BQT > 0 ? BQT : 8];
#pragma unroll
      for (int t = 0; t < (BQT > 0 ? BQT : 8); ++t) acc[t] = 0;
      int pop = 0;
#pragma unroll
      for (int w = 0; w < WR; ++w) {
        if (w < W) {
          const uint32_t c = f.cw[w];
          pop += __popc(c);
#pragma unroll
          for (int t = 0; t < (BQT > 0 ? BQT : 8); ++t)
            if (t < BQ)
              acc[t] += __popc(c & (PR > 1 ? f.pl[(w * (BQT > 0 ? BQT : 1) + t) % PR] : planes[w * bqs + t]));
        }
      }
      int ip = 0;
#pragma unroll
      for (int t = 0; t < (BQT > 0 ? BQT : 8); ++t)
        if (t < BQ) ip += acc[t] << t;
      const float est =
          rbq_estimate(f.sc.x, f.sc.y, f.sc.z, -(int)f.sc.w, ip, f.fa, f.fm, rbq_vx(f.fm, pop, D));
      const int v = (f.mb << 6) + lane;
      const bool pass = v < f.len && ord_f32(est) <= s_thr;
      const uint64_t m = __ballot(pass);
      if (m) {
        uint32_t base = 0;
        if (lane == 0) base = (uint32_t)fill + atomicAdd(&s_cnt[par], (uint32_t)__popcll(m));
        base = __shfl(base, 0);
        if (pass) buf[base + lane_prefix(m)] = key64(est, (uint32_t)f.id);
      }
    };
    // round r: wave w takes micro-block r * NW + w, from register set r % 2,
    // which is then refilled with the micro-block two rounds on. Round r
    // appends behind the fill through counter s_cnt[r % 3]; the counter of
    // round r + 1 is cleared during round r (its last readers, after round
    // r - 2's barrier, are all past round r - 1's), so one barrier per round
    // gives every thread the same fill.
    FusedSlot<WR, PR> A, B;
    auto round = [&](int idx, FusedSlot<WR, PR>& f) __attribute__((always_inline)) {
      const int par = rr % 3;
      if (tid == 0) s_cnt[(rr + 1) % 3] = 0u;
      if (idx < total) {
        scan(f, par);
        if (idx + 2 * NW < total) load(idx + 2 * NW, f);
      }
      __syncthreads();
      fill += (int)s_cnt[par];
      ++rr;
      if (fill > a.cap - NT) shrink();  // the next round could overflow
    };
    if (wave < total) load(wave, A);
    if (NW + wave < total) load(NW + wave, B);
    for (int b0 = 0; b0 < total; b0 += 2 * NW) {
      round(b0 + wave, A);
      round(b0 + NW + wave, B);
    }
    __syncthreads();
  }
  if (fill > Rq) shrink();
  const int keep = min(fill, Rq);
  for (int r = tid; r < Rq; r += NT) row[r] = r < keep ? buf[r] : KEY_NONE;
  // s_thr is the R-th estimate of the last selection (the kept keys' R-th when
  // the buffer ended above Rq), else the threshold the query came with: an
  // upper bound on its R-th estimate either way
  if (tid == 0) {
    if (a.reset)
      a.qthr[i] = s_thr;  // (this workgroup alone handles query i)
    else
      atomicMin(&a.qthr[i], s_thr);
  }
}

template <int WT, int BQT>
static void fused_dispatch(hipStream_t s, const FusedArgs& a, size_t lds) {
  static std::once_flag once;  // (static and dynamic LDS together exceed 64 KB)
  std::call_once(once, [lds] {
    RBQ_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(k_scan_fused<WT, BQT>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  });
  hipLaunchKernelGGL((k_scan_fused<WT, BQT>), dim3(a.nq), dim3(kFusedNT), lds, s, a);
}

void launch_scan_fused(hipStream_t s, FusedArgs a) {
  if (a.nq <= 0 || a.pn <= 0) return;
  a.cap = kFusedCap;
  RBQ_CHECK(a.R + kFusedNT <= a.cap - kFusedNT, "fused scan: rerank_n too large for its LDS buffer");
  RBQ_CHECK(a.L.W <= 32, "fused scan supports d <= 1024");
  const size_t lds = (size_t)a.cap * sizeof(uint64_t);
  const int bq4 = a.Q.bqs == 4;
  if (bq4 && a.L.W == 4)
    fused_dispatch<4, 4>(s, a, lds);
  else if (bq4 && a.L.W == 3)
    fused_dispatch<3, 4>(s, a, lds);
  else if (bq4 && a.L.W == 2)
    fused_dispatch<2, 4>(s, a, lds);
  else
    fused_dispatch<0, 0>(s, a, lds);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Exact re-rank (Phase 5 on the GPU): per query, the R candidates' raw vectors
// are gathered (16 lanes per candidate, float4 loads, four candidates per wave
// in flight), ||q - x||^2 is summed in FP32, and the k best (distance, id)
// keys are selected by an MSB-first radix select and sorted.
// ---------------------------------------------------------------------------

// The k smallest of n 64-bit keys held in LDS (whole workgroup): after the
// call, sel[0..k) holds them ascending. hist: 256 words, wsum: 4 words,
// sel: KP = pow2 >= k keys.
__device__ void lds_select_sorted(const uint64_t* keys, int n, int k, int KP, uint64_t* sel,
                                  uint32_t* hist, uint32_t* wsum, uint32_t* s_misc) {
  const int tid = threadIdx.x;
  uint64_t prefix = 0, pmask = 0;
  uint32_t rem = (uint32_t)k;
  const bool take_all = n <= k;
  if (!take_all) {
    for (int shift = 56; shift >= 0; shift -= 8) {
      hist[tid] = 0;
      __syncthreads();
      for (int c = tid; c < n; c += 256) {
        const uint64_t key = keys[c];
        if ((key & pmask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
      }
      __syncthreads();
      const uint32_t h = hist[tid];
      const uint32_t incl = block_incl_scan_256(h, wsum);
      const uint32_t excl = incl - h;
      if (excl < rem && rem <= incl) {
        s_misc[0] = (uint32_t)tid;
        s_misc[1] = rem - excl;
        s_misc[2] = h;
      }
      __syncthreads();
      prefix |= (uint64_t)s_misc[0] << shift;
      pmask |= 0xFFull << shift;
      rem = s_misc[1];
      const uint32_t bucket = s_misc[2];
      __syncthreads();
      if (bucket == rem) break;
    }
  }
  if (tid == 0) s_misc[3] = 0;
  __syncthreads();
  if (take_all) {
    for (int c = tid; c < n; c += 256) sel[atomicAdd(&s_misc[3], 1u)] = keys[c];
  } else {
    for (int c = tid; c < n; c += 256)
      if (keys[c] < prefix) sel[atomicAdd(&s_misc[3], 1u)] = keys[c];
    __syncthreads();
    const uint64_t hi = prefix | ~pmask;
    for (int c = tid; c < n; c += 256) {
      const uint64_t key = keys[c];
      if (key >= prefix && key <= hi) {
        const uint32_t p = atomicAdd(&s_misc[3], 1u);
        if (p < (uint32_t)k) sel[p] = key;
      }
    }
  }
  __syncthreads();
  const int cnt = min((int)s_misc[3], k);
  for (int i = cnt + tid; i < KP; i += 256) sel[i] = KEY_NONE;
  __syncthreads();
  bitonic_sort_lds(sel, KP);
}

// Four consecutive elements of a raw-vector row as floats (FP32 rows, or
// byte rows holding integers 0..255 exactly).
__device__ inline float4 row4(const float* __restrict__ X, size_t e) {
  return *reinterpret_cast<const float4*>(X + e);
}
__device__ inline float4 bytes4(uint32_t w) {
  return make_float4((float)(w & 0xFFu), (float)((w >> 8) & 0xFFu), (float)((w >> 16) & 0xFFu),
                     (float)(w >> 24));
}
__device__ inline float4 row4(const uint8_t* __restrict__ X, size_t e) {
  return bytes4(*reinterpret_cast<const uint32_t*>(X + e));
}
// Sixteen consecutive elements (four groups of four) starting at element e,
// of which the first `ng` groups are read (the rest are zero). Byte rows whose
// starts are 16-byte aligned take one 16-byte load.
__device__ inline void row16(const float* __restrict__ X, size_t e, int ng, bool, float4 (&x)[4]) {
#pragma unroll
  for (int j = 0; j < 4; ++j) x[j] = j < ng ? row4(X, e + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
}
__device__ inline void row16(const uint8_t* __restrict__ X, size_t e, int ng, bool a16, float4 (&x)[4]) {
  if (a16 && ng >= 4) {
    const uint4 w = *reinterpret_cast<const uint4*>(X + e);
    x[0] = bytes4(w.x);
    x[1] = bytes4(w.y);
    x[2] = bytes4(w.z);
    x[3] = bytes4(w.w);
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = j < ng ? row4(X, e + 4 * j) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_rerank(const float* __restrict__ q, int ldq,
                                                const T* __restrict__ X, int64_t n, int ldx, int d,
                                                const uint64_t* __restrict__ cand, int64_t ldc,
                                                int R, int k, int KP, int64_t* __restrict__ ids,
                                                float* __restrict__ dist,
                                                const int32_t* __restrict__ rowk) {
  // [R] candidate keys, then [KP] selection keys; KP < 0 means no separate
  // selection buffer: ck holds -KP (pow2 >= R) keys and is sorted in place
  extern __shared__ uint64_t ck[];
  uint64_t* sel = ck + (KP > 0 ? R : -KP);
  float4* qs = reinterpret_cast<float4*>(sel + (KP > 0 ? KP : 0));  // the query, ldx/4 float4
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t s_misc[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i = blockIdx.x;
  const int kr = rowk ? rowk[i] : k;  // this row's k (<= k)
  const int nf4 = ldx >> 2;
  for (int t = tid; t < nf4; t += 256)
    qs[t] = (t * 4 < d) ? reinterpret_cast<const float4*>(q + i * ldq)[t] : make_float4(0, 0, 0, 0);
  for (int c = tid; c < R; c += 256) ck[c] = cand[i * ldc + c];  // the keys, coalesced
  __syncthreads();
  // 8 lanes per candidate (a lane takes 16 consecutive elements of every 128),
  // RU candidates per slot in flight: in round r, wave w, slot s takes
  // candidates 32 (RU r + u) + 8 w + s; each slot rewrites only its own keys.
  // Byte and FP32 rows are summed in the same order.
  constexpr int RU = 4;
  const int sub8 = lane >> 3, sl8 = lane & 7;
  const bool a16 = (ldx * sizeof(T)) % 16 == 0;
  for (int c0 = 0; c0 < R; c0 += 32 * RU) {
    uint64_t key[RU];
    size_t row[RU];
    bool ok[RU];
    float acc[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int c = c0 + 32 * u + 8 * wave + sub8;
      key[u] = c < R ? ck[c] : KEY_NONE;
      ok[u] = key[u] != KEY_NONE && (int64_t)(uint32_t)key[u] < n;  // ids outside [0, n) are never read
      row[u] = ok[u] ? (size_t)(uint32_t)key[u] * ldx : 0;
      acc[u] = 0.f;
    }
    for (int f0 = 4 * sl8; f0 < nf4; f0 += 32) {
      const int ng = min(4, nf4 - f0);
      float4 qv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) qv[j] = j < ng ? qs[f0 + j] : make_float4(0.f, 0.f, 0.f, 0.f);
      float4 xv[RU][4];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        if (ok[u]) {
          row16(X, row[u] + 4 * (size_t)f0, ng, a16, xv[u]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) xv[u][j] = qv[j];
        }
      }
#pragma unroll
      for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float a0 = qv[j].x - xv[u][j].x, a1 = qv[j].y - xv[u][j].y, a2 = qv[j].z - xv[u][j].z,
                      a3 = qv[j].w - xv[u][j].w;
          acc[u] += a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3;
        }
    }
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      for (int off = 4; off > 0; off >>= 1) acc[u] += __shfl_xor(acc[u], off);
      const int c = c0 + 32 * u + 8 * wave + sub8;
      if (sl8 == 0 && c < R) ck[c] = ok[u] ? key64(acc[u], (uint32_t)key[u]) : KEY_NONE;
    }
  }
  __syncthreads();
  if (KP > 0) {
    lds_select_sorted(ck, R, kr, KP, sel, hist, wsum, s_misc);
  } else {  // large k: sort all candidates in place (ck holds pow2 >= R keys)
    const int KR = -KP;
    for (int t = R + tid; t < KR; t += 256) ck[t] = KEY_NONE;
    __syncthreads();
    bitonic_sort_lds(ck, KR);
    sel = ck;
  }
  for (int r = tid; r < k; r += 256) {
    const uint64_t v = r < kr ? sel[r] : KEY_NONE;
    ids[i * k + r] = v == KEY_NONE ? -1 : (int64_t)(uint32_t)v;
    dist[i * k + r] = v == KEY_NONE ? INFINITY : f32_ord((uint32_t)(v >> 32));
  }
}

template <typename T>
static void rerank_impl(hipStream_t s, const float* q, int ldq, const T* X, int64_t n, int ldx,
                        int d, const uint64_t* cand, int64_t ldc, int nq, int R, int k, int64_t* ids,
                        float* dist, const int32_t* rowk) {
  if (nq <= 0) return;
  RBQ_CHECK(ldx % 4 == 0 && ldq % 4 == 0, "rows must be padded to 4 floats");
  int KP = pow2_at_least(k);
  size_t lds = (size_t)(R + KP) * sizeof(uint64_t) + (size_t)ldx * sizeof(float);
  if (lds > (size_t)(60 << 10)) {
    KP = -pow2_at_least(R);
    lds = (size_t)(-KP) * sizeof(uint64_t) + (size_t)ldx * sizeof(float);
  }
  RBQ_CHECK(lds <= (size_t)(64 << 10), "re-rank needs too much LDS for this d and rerank_n");
  hipLaunchKernelGGL(k_rerank<T>, dim3(nq), dim3(256), lds, s, q, ldq, X, n, ldx, d, cand, ldc, R, k,
                     KP, ids, dist, rowk);
  RBQ_HIP(hipGetLastError());
}

void launch_rerank(hipStream_t s, const float* q, int ldq, const float* X, int64_t n, int ldx,
                   int d, const uint64_t* cand, int64_t ldc, int nq, int R, int k, int64_t* ids,
                   float* dist, const int32_t* rowk) {
  rerank_impl(s, q, ldq, X, n, ldx, d, cand, ldc, nq, R, k, ids, dist, rowk);
}

void launch_rerank_u8(hipStream_t s, const float* q, int ldq, const uint8_t* X, int64_t n, int ldx,
                      int d, const uint64_t* cand, int64_t ldc, int nq, int R, int k, int64_t* ids,
                      float* dist, const int32_t* rowk) {
  rerank_impl(s, q, ldq, X, n, ldx, d, cand, ldc, nq, R, k, ids, dist, rowk);
}

// Raw vectors that are all integers in [0, 255] (e.g. SIFT-style descriptors
// stored as FP32) can be held as bytes without changing any value.
__global__ void k_count_not_u8(const float* X, int64_t rows, int d, int ld, unsigned* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = rows * d;
  unsigned bad = 0;
  for (int64_t e = t; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / d;
    const float v = X[r * ld + (e - r * d)];
    bad += !(v >= 0.f && v <= 255.f && v == rintf(v));
  }
  if (bad) atomicAdd(out, bad);
}

__global__ void k_to_u8(const float* X, int64_t total, uint8_t* out) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x)
    out[e] = (uint8_t)X[e];
}

void launch_count_not_u8(hipStream_t s, const float* X, int64_t rows, int d, int ld, unsigned* out) {
  hipLaunchKernelGGL(k_count_not_u8, dim3(1024), dim3(256), 0, s, X, rows, d, ld, out);
  RBQ_HIP(hipGetLastError());
}

void launch_to_u8(hipStream_t s, const float* X, int64_t total, uint8_t* out) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_to_u8, dim3(2048), dim3(256), 0, s, X, total, out);
  RBQ_HIP(hipGetLastError());
}

__global__ void k_mask_probes(int32_t* probes, int nq, int nprobe, const int32_t* qnp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nq * nprobe) return;
  const int64_t i = t / nprobe;
  if ((int)(t - i * nprobe) >= qnp[i]) probes[t] = -1;
}

void launch_mask_probes(hipStream_t s, int32_t* probes, int nq, int nprobe, const int32_t* qnp) {
  const int64_t n = (int64_t)nq * nprobe;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mask_probes, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, probes, nq,
                     nprobe, qnp);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// RaBitQ encoder (Sec. 3.1.1 Phase 3, Sec. 3.2.2) in FP64: one workgroup per
// micro-block of 64 list positions. The residual norm n_x is taken from
// r = x - c directly (an orthogonal P preserves it, so it need not wait for
// the rotation); z = P^T r; code bit = [z >= 0]; alpha = ||z||_1/(sqrt(D) n_x).
// Writes the micro-block record (codes, n_x^2, -2 n_x/(sqrt(D) alpha)) and the
// unfolded (n_x, alpha) for export.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_encode(const float* __restrict__ X, int ldx,
                                                const float* __restrict__ C, int ldc,
                                                const float* __restrict__ Pt, int ldp,
                                                const int32_t* __restrict__ pos2id,
                                                const int32_t* __restrict__ mb_list, int64_t mb_begin,
                                                int d, int W, uint32_t* __restrict__ blocks,
                                                float* __restrict__ nx_out,
                                                float* __restrict__ alpha_out) {
  extern __shared__ uint32_t bits[];          // [W][64]
  __shared__ double rs[64][33];
  __shared__ double part[4][64];
  __shared__ double l1part[4][64];
  const int tid = threadIdx.x;
  const int v = tid & 63;
  const int g = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t mb = mb_begin + blockIdx.x;
  const int j = mb_list[mb];
  const float* cj = C + (int64_t)j * ldc;
  for (int t = tid; t < W * 64; t += 256) bits[t] = 0u;
  {  // ||x - c||^2 in FP64, four interleaved partial sums per vector
    const int id = pos2id[mb * 64 + v];
    double s2 = 0.0;
    if (id >= 0) {
      const float* x = X + (int64_t)id * ldx;
      for (int t = g; t < d; t += 4) {
        const double r = (double)x[t] - (double)cj[t];
        s2 += r * r;
      }
    }
    part[g][v] = s2;
  }
  double l1 = 0.0;
  const int lr = tid >> 2, lc = (tid & 3) * 8;
  const int idl = pos2id[mb * 64 + lr];
  for (int i0 = 0; i0 < d; i0 += 128) {
    double acc[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) acc[t] = 0.0;
    for (int d0 = 0; d0 < d; d0 += 32) {
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dd = d0 + lc + c;
        double r = 0.0;
        if (idl >= 0 && dd < d) r = (double)X[(int64_t)idl * ldx + dd] - (double)cj[dd];
        rs[lr][lc + c] = r;
      }
      __syncthreads();
      const int dmax = min(32, d - d0);
      for (int dd = 0; dd < dmax; ++dd) {
        const double rv = rs[v][dd];
#pragma unroll
        for (int t = 0; t < 32; ++t) {
          const int oi = i0 + g + 4 * t;
          if (oi < d) acc[t] += rv * (double)Pt[(int64_t)oi * ldp + d0 + dd];
        }
      }
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int oi = i0 + g + 4 * t;
      if (oi < d) {
        if (acc[t] >= 0.0) atomicOr(&bits[(oi >> 5) * 64 + v], 1u << (oi & 31));
        l1 += fabs(acc[t]);
      }
    }
  }
  l1part[g][v] = l1;
  __syncthreads();
  const int64_t pos = mb * 64 + v;
  const int id = pos2id[pos];
  const size_t rec = (size_t)(W + 2) * 64;
  uint32_t* out = blocks + mb * rec;
  for (int t = tid; t < W * 64; t += 256) {
    const int vv = t & 63;
    out[t] = pos2id[mb * 64 + vv] >= 0 ? bits[t] : 0u;
  }
  if (g == 0) {
    float fadd = INFINITY, fmul = 0.f, nxf = 0.f, alf = 1.f;
    if (id >= 0) {
      const double n2 = part[0][v] + part[1][v] + part[2][v] + part[3][v];
      const double nx = sqrt(n2);
      const double L1 = l1part[0][v] + l1part[1][v] + l1part[2][v] + l1part[3][v];
      const double alpha = nx > 0.0 ? L1 / (sqrt((double)d) * nx) : 1.0;
      fadd = (float)(nx * nx);
      fmul = (float)(-2.0 * nx / (sqrt((double)d) * alpha));
      nxf = (float)nx;
      alf = (float)alpha;
    }
    out[W * 64 + v] = __float_as_uint(fadd);
    out[(W + 1) * 64 + v] = __float_as_uint(fmul);
    nx_out[pos] = nxf;
    alpha_out[pos] = alf;
  }
}

void launch_encode(hipStream_t s, const float* X, int ldx, const float* C, int ldc, const float* Pt,
                   int ldp, const int32_t* pos2id, const int32_t* mb_list, int64_t mb_begin,
                   int64_t mb_end, int d, int W, uint32_t* blocks, float* nx_out,
                   float* alpha_out) {
  const int64_t n = mb_end - mb_begin;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_encode, dim3((unsigned)n), dim3(256), (size_t)W * 64 * sizeof(uint32_t), s,
                     X, ldx, C, ldc, Pt, ldp, pos2id, mb_list, mb_begin, d, W, blocks, nx_out,
                     alpha_out);
  RBQ_HIP(hipGetLastError());
}

__global__ void k_rotate_rows_f64(const float* __restrict__ A, int lda, const float* __restrict__ Pt,
                                  int ldp, int rows, int d, float* __restrict__ out, int ldo,
                                  float* __restrict__ nrm) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)rows * d) return;
  const int64_t r = t / d;
  const int i = (int)(t - r * d);
  const float* a = A + r * lda;
  const float* p = Pt + (int64_t)i * ldp;
  double acc = 0.0;
  for (int k = 0; k < d; ++k) acc += (double)a[k] * (double)p[k];
  out[r * ldo + i] = (float)acc;
  if (nrm && i == 0) {
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)a[k] * (double)a[k];
    nrm[r] = (float)s;
  }
}

void launch_rotate_rows_f64(hipStream_t s, const float* A, int lda, const float* Pt, int ldp,
                            int rows, int d, float* out, int ldo, float* nrm) {
  const int64_t n = (int64_t)rows * d;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_rotate_rows_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A, lda,
                     Pt, ldp, rows, d, out, ldo, nrm);
  RBQ_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Small utility kernels.
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}
__global__ void k_fill_u64(uint64_t* p, uint64_t v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = v;
}
// p[r * ld + c] = v for r < rows, c < cols
__global__ void k_fill_rows_u64(uint64_t* p, int64_t ld, int64_t rows, int cols, uint64_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * cols) return;
  const int64_t r = t / cols;
  p[r * ld + (t - r * cols)] = v;
}
void launch_fill_rows_u64(hipStream_t s, uint64_t* p, int64_t ld, int64_t rows, int cols, uint64_t v) {
  const int64_t n = rows * cols;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_rows_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, ld, rows,
                     cols, v);
  RBQ_HIP(hipGetLastError());
}

// A search's per-query state in one launch: candidate rows empty, thresholds
// open, pool fills and overflow flags zero, the extra words cleared or set.
__global__ void k_search_init(SearchInit a) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t cells = (int64_t)a.nq * a.R;
  for (int64_t t = t0; t < cells; t += step) {
    const int64_t r = t / a.R;
    a.cand[r * a.cand_ld + (t - r * a.R)] = KEY_NONE;
  }
  for (int64_t t = t0; t < a.nq; t += step) {
    a.qthr[t] = 0xFFFFFFFFu;
    a.pcnt[t] = 0u;
    if (a.overflow) a.overflow[t] = 0u;
  }
  for (int64_t t = t0; t < a.n0; t += step) a.z0[t] = 0u;
  for (int64_t t = t0; t < a.n2; t += step) a.f2[t] = 0xFFFFFFFFu;
}
void launch_search_init(hipStream_t s, const SearchInit& a) {
  const int64_t n = std::max<int64_t>({(int64_t)a.nq * a.R, a.nq, a.n0, a.n2});
  if (n <= 0) return;
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
  hipLaunchKernelGGL(k_search_init, dim3((unsigned)blocks), dim3(256), 0, s, a);
  RBQ_HIP(hipGetLastError());
}

void launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  RBQ_HIP(hipGetLastError());
}
void launch_fill_u64(hipStream_t s, uint64_t* p, uint64_t v, int64_t n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
  RBQ_HIP(hipGetLastError());
}

__global__ void k_gather_rows(const float* __restrict__ X, int ldx, const int64_t* __restrict__ idx,
                              int64_t n, float* __restrict__ out, int ldo) {
  const int64_t r = blockIdx.x;
  if (r >= n) return;
  const float* src = X + idx[r] * ldx;
  for (int t = threadIdx.x; t < ldo; t += blockDim.x) out[r * ldo + t] = src[t];
}
void launch_gather_rows(hipStream_t s, const float* X, int ldx, const int64_t* idx, int64_t n,
                        float* out, int ldo) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)n), dim3(128), 0, s, X, ldx, idx, n, out, ldo);
  RBQ_HIP(hipGetLastError());
}

// k-means++ seeding on the device. mind[t] holds the squared distance of row t
// to its nearest chosen centre; blocksum[b] the FP64 sum of mind over rows
// [256 b, 256 b + 256). One wave per row: lanes stride the dimensions, so every
// load instruction reads one contiguous span of the row.
__global__ __launch_bounds__(256) void k_kpp_update(const float* __restrict__ T, int ldt, int64_t n,
                                                    int d, const int64_t* __restrict__ pick,
                                                    float* __restrict__ mind,
                                                    double* __restrict__ blocksum, int first) {
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const float* c = T + (*pick) * ldt;
  double part = 0.0;
  for (int rr = 0; rr < 64; ++rr) {
    const int64_t t = (int64_t)blockIdx.x * 256 + wave * 64 + rr;
    if (t >= n) break;
    const float* x = T + t * ldt;
    float acc = 0.f;
    for (int k = lane; k < d; k += 64) {
      const float df = x[k] - c[k];
      acc += df * df;
    }
    acc = wave_sum(acc);
    const float m = first ? acc : fminf(mind[t], acc);
    if (lane == 0) mind[t] = m;
    part += (double)m;
  }
  if (lane == 0) red[wave] = part;
  __syncthreads();
  if (threadIdx.x == 0) blocksum[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

void launch_kpp_update(hipStream_t s, const float* T, int ldt, int64_t n, int d, const int64_t* pick,
                       float* mind, double* blocksum, int first) {
  hipLaunchKernelGGL(k_kpp_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, T, ldt, n, d,
                     pick, mind, blocksum, first);
  RBQ_HIP(hipGetLastError());
}

// Samples row t with probability mind[t] / sum(mind): locates u * total in the
// running sums (blocks first, then rows inside the block), in a fixed order.
__global__ __launch_bounds__(256) void k_kpp_choose(const float* __restrict__ mind,
                                                    const double* __restrict__ blocksum, int64_t n,
                                                    double u, int64_t* __restrict__ pick) {
  __shared__ double part[256];
  __shared__ double pre[257];
  const int tid = threadIdx.x;
  const int64_t nb = (n + 255) / 256;
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = tid * per, b1 = min(nb, b0 + per);
  double s = 0.0;
  for (int64_t b = b0; b < b1; ++b) s += blocksum[b];
  part[tid] = s;
  __syncthreads();
  if (tid == 0) {
    pre[0] = 0.0;
    for (int t = 0; t < 256; ++t) pre[t + 1] = pre[t] + part[t];
    const double total = pre[256];
    int64_t choice = 0;
    if (!(total > 0.0)) {
      choice = min(n - 1, (int64_t)(u * (double)n));
    } else {
      const double target = u * total;
      int t = 0;
      while (t < 255 && pre[t + 1] <= target) ++t;
      double acc = pre[t];
      int64_t b = min((int64_t)t * per, nb - 1);
      const int64_t bend = min(nb, b + per);
      while (b + 1 < bend && acc + blocksum[b] <= target) acc += blocksum[b++];
      int64_t r = b * 256;
      const int64_t rend = min(n, r + 256);
      while (r + 1 < rend && acc + (double)mind[r] <= target) acc += (double)mind[r++];
      // never pick a row whose weight is zero
      while (r < rend - 1 && mind[r] == 0.f) ++r;
      choice = min(r, n - 1);
    }
    *pick = choice;
  }
}

void launch_kpp_choose(hipStream_t s, const float* mind, const double* blocksum, int64_t n, double u,
                       int64_t* pick) {
  hipLaunchKernelGGL(k_kpp_choose, dim3(1), dim3(256), 0, s, mind, blocksum, n, u, pick);
  RBQ_HIP(hipGetLastError());
}

__global__ void k_copy_row(const float* __restrict__ T, int ldt, const int64_t* __restrict__ pick,
                           float* __restrict__ dst, int d) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d) dst[t] = T[(*pick) * ldt + t];
}
void launch_copy_row(hipStream_t s, const float* T, int ldt, const int64_t* pick, float* dst, int d) {
  hipLaunchKernelGGL(k_copy_row, dim3((d + 255) / 256), dim3(256), 0, s, T, ldt, pick, dst, d);
  RBQ_HIP(hipGetLastError());
}

}  // namespace rbq
