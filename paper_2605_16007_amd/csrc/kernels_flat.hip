// IVF-Flat scan on the FP32 matrix cores: the comparison system of Sec. 4.2
// (full-precision vectors in the probed lists, Sec. 2.1.2), built the same
// list-major way as the code scan so that the two are compared on equal
// footing on one GPU.
//
// Layout: every list's vectors in 64-vector micro-blocks (the code blocks'
// numbering), each block a record of Dp = round_up(d, 4) rows of 64 floats
// (dimension-major, so a wave reads a row as one 256-byte line) and one row of
// FP32 squared norms ||x||^2 (+inf in padding lanes). An item is one list and
// up to 32 of the queries that probe it; per 16 vectors x 16 queries the
// products <q, x> are v_mfma_f32_16x16x4_f32 over the dimensions, and
//   d^2 = ||q||^2 + ||x||^2 - 2 <q, x>
// is tested against the query's threshold. Survivors go to the query's pool
// as (d^2, id) keys; the search's merges keep the best rerank_n and its exact
// re-rank (direct differences) orders them, so the returned distances are the
// same exact ones as IVF-RaBitQ's.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace rbq {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int FG = 32;         // queries per item (two 16-query tiles)
constexpr int FDMAX = 256;     // dimensions held in LDS per query
constexpr int FSTAGE = 512;    // survivors staged per wave before a flush

__device__ inline uint32_t lane_prefix_f(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// ||x||^2 rows and the dimension-major rows of every micro-block.
__global__ void k_flat_fill(const float* __restrict__ X, int ldx, const int32_t* __restrict__ pos2id,
                            int64_t mb_begin, int d, int dp, float* __restrict__ out) {
  const int64_t mb = mb_begin + blockIdx.x;
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;  // 4 waves split the rows
  const int id = pos2id[mb * 64 + lane];
  float* rec = out + mb * (int64_t)(dp + 1) * 64;
  for (int r = part; r < dp; r += 4)
    rec[(int64_t)r * 64 + lane] = (id >= 0 && r < d) ? X[(int64_t)id * ldx + r] : 0.f;
  if (part == 0) {
    double s = 0.0;
    if (id >= 0)
      for (int r = 0; r < d; ++r) {
        const double v = X[(int64_t)id * ldx + r];
        s += v * v;
      }
    rec[(int64_t)dp * 64 + lane] = id >= 0 ? (float)s : INFINITY;
  }
}

// DP: the largest row count the instance handles; the records have
// dp = round_up(d, 4) rows (dp <= DP)
template <int DP>
__global__ __launch_bounds__(256) void k_scan_flat(FlatArgs a) {
  constexpr int S = DP / 4;                 // k steps of 4 dimensions, at most
  __shared__ float sQv[FG][DP + 1];         // the item's queries (+1: no bank conflicts)
  __shared__ float sQn[FG], sThr[FG];
  __shared__ int32_t sQ[FG];
  __shared__ uint64_t sStage[4][FSTAGE];
  __shared__ uint32_t sFcnt[4][FG], sFbase[4][FG];
  __shared__ int32_t sItem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int d = a.d;
  const int dp = (d + 3) & ~3;
  const int ns = dp >> 2;  // k steps of this index
  int stage_n = 0;
  int list_pos0 = 0;
  // moves the staged survivors to their queries' pools (one global atomic
  // per query slot, ids looked up lane-parallel)
  auto flush = [&](int nst) {
    if (nst == 0) return;
    if (lane < FG) sFcnt[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) atomicAdd(&sFcnt[wave][(uint32_t)sStage[wave][e] >> 26], 1u);
    __builtin_amdgcn_wave_barrier();
    if (lane < FG) {
      const uint32_t c = sFcnt[wave][lane];
      sFbase[wave][lane] = c ? atomicAdd(&a.pcnt[sQ[lane]], c) : 0u;
      sFcnt[wave][lane] = 0u;
    }
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) {
      const uint64_t kp = sStage[wave][e];
      const uint32_t lo = (uint32_t)kp;
      const int q = (int)(lo >> 26);
      const int qi = sQ[q];
      const uint32_t slot = sFbase[wave][q] + atomicAdd(&sFcnt[wave][q], 1u);
      const int id = a.pos2id[list_pos0 + (int)(lo & 0x3FFFFFFu)];
      const uint64_t key = ((uint64_t)ord_f32(__uint_as_float((uint32_t)(kp >> 32))) << 32) | (uint32_t)id;
      if (slot < (uint32_t)a.cap) {
        a.pool[(int64_t)qi * a.pool_ld + a.R + slot] = key;
      } else {
        a.overflow[qi] = 1u;
        *a.any_overflow = 1u;
      }
    }
    __builtin_amdgcn_wave_barrier();
  };
  const int first_item = a.item_off[0], end_item = a.item_off[1];
  const int64_t rec = (int64_t)(dp + 1) * 64;
  for (;;) {
    if (tid == 0) sItem = first_item + (int32_t)atomicAdd(a.item_counter, 1u);
    __syncthreads();
    const int item = sItem;
    __syncthreads();
    if (item >= end_item) break;
    const int4 it = a.items[item];
    const int first = it.y, count = it.z;
    const int nt = (count + 15) >> 4;
    const int mb0 = it.x, len = it.w;
    const int nmb = (len + 63) >> 6;
    list_pos0 = mb0 << 6;
    // the item's queries, their squared norms (fixed order) and thresholds
    for (int e = tid; e < FG * DP; e += 256) {
      const int q = e / DP, c = e - q * DP;
      float v = 0.f;
      if (q < count && c < d) {
        const int qi = a.slots[first + q] / a.nprobe;
        v = a.q[(int64_t)qi * a.ldq + c];
      }
      sQv[q][c] = v;
    }
    if (tid < FG) {
      if (tid < count) {
        const int qi = a.slots[first + tid] / a.nprobe;
        sQ[tid] = qi;
        const uint32_t th = a.qthr[qi];
        sThr[tid] = th == 0xFFFFFFFFu ? INFINITY : f32_ord(th);
      } else {
        sQ[tid] = 0;
        sThr[tid] = NAN;  // an empty slot never passes
      }
    }
    __syncthreads();
    if (tid < FG) {
      float s = 0.f;
      for (int c = 0; c < d; ++c) s = fmaf(sQv[tid][c], sQv[tid][c], s);
      sQn[tid] = s;
    }
    __syncthreads();
    const int lg = lane >> 4, lr = lane & 15;
    float qn[2], thr[2];
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      qn[n] = sQn[16 * n + lr];
      thr[n] = sThr[16 * n + lr];
    }
    for (int mb = wave; mb < nmb; mb += 4) {
      const float* blk = a.blocks + (int64_t)(mb0 + mb) * rec;
#pragma unroll 1
      for (int m = 0; m < 4; ++m) {
        // A: vectors 16 m + lr, dimensions 4 s + lg (one float per lane)
        float A[S];
#pragma unroll
        for (int s = 0; s < S; ++s) A[s] = s < ns ? blk[(int64_t)(4 * s + lg) * 64 + 16 * m + lr] : 0.f;
        v4f acc[2];
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          acc[n] = v4f{0.f, 0.f, 0.f, 0.f};
          if (n < nt) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
              if (s < ns)  // (uniform)
                acc[n] = __builtin_amdgcn_mfma_f32_16x16x4f32(A[s], sQv[16 * n + lr][4 * s + lg], acc[n], 0, 0, 0);
            }
          }
        }
        // this lane's result rows: vectors 16 m + 4 lg + r, column lr
        const float4 xn4 = *reinterpret_cast<const float4*>(blk + (int64_t)dp * 64 + 16 * m + 4 * lg);
        const float xn[4] = {xn4.x, xn4.y, xn4.z, xn4.w};
        const uint32_t rel0 = (uint32_t)((mb << 6) + 16 * m + 4 * lg);
#pragma unroll
        for (int n = 0; n < 2; ++n) {
          if (n >= nt) break;
          const uint32_t tag = rel0 | ((uint32_t)(16 * n + lr) << 26);
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float d2 = fmaf(-2.f, acc[n][r], qn[n] + xn[r]);
            const bool pass = d2 <= thr[n];  // +inf padding and NaN slots never pass
            const uint64_t me = __builtin_amdgcn_ballot_w64(pass);
            if (pass) {
              const uint32_t e = __builtin_amdgcn_mbcnt_hi((uint32_t)(me >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((uint32_t)me, (uint32_t)stage_n));
              sStage[wave][e] = ((uint64_t)__float_as_uint(d2) << 32) | (tag + (uint32_t)r);
            }
            stage_n += (int)__popcll(me);
          }
          if (stage_n > FSTAGE - 256) {
            __builtin_amdgcn_wave_barrier();
            flush(stage_n);
            stage_n = 0;
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    flush(stage_n);
    stage_n = 0;
    __syncthreads();  // the item's LDS is restaged for the next one
  }
}

}  // namespace

int flat_dp(int d) { return (int)round_up(d, 4); }

void launch_flat_fill(hipStream_t s, const float* X, int ldx, const int32_t* pos2id, int64_t nmb, int d,
                      float* out) {
  const int dp = flat_dp(d);
  for (int64_t m0 = 0; m0 < nmb; m0 += 65535) {
    const unsigned g = (unsigned)std::min<int64_t>(65535, nmb - m0);
    hipLaunchKernelGGL(k_flat_fill, dim3(g), dim3(256), 0, s, X, ldx, pos2id, m0, d, dp, out);
    RBQ_HIP(hipGetLastError());
  }
}

void launch_scan_flat(hipStream_t s, const FlatArgs& a, int workgroups) {
  RBQ_CHECK(a.G >= 1 && a.G <= FG, "IVF-Flat items hold at most 32 queries");
  const int dp = flat_dp(a.d);
  RBQ_CHECK(dp <= FDMAX, "the IVF-Flat scan supports d <= 256");
  if (dp <= 32)
    hipLaunchKernelGGL(k_scan_flat<32>, dim3(workgroups), dim3(256), 0, s, a);
  else if (dp <= 64)
    hipLaunchKernelGGL(k_scan_flat<64>, dim3(workgroups), dim3(256), 0, s, a);
  else if (dp <= 96)
    hipLaunchKernelGGL(k_scan_flat<96>, dim3(workgroups), dim3(256), 0, s, a);
  else if (dp <= 128)
    hipLaunchKernelGGL(k_scan_flat<128>, dim3(workgroups), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(k_scan_flat<256>, dim3(workgroups), dim3(256), 0, s, a);
  RBQ_HIP(hipGetLastError());
}

}  // namespace rbq
