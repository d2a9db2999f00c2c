// List-major code scan on int8 MFMA (gfx950) for batches in which many
// queries probe the same list.
//
// The query-major scan reads a list once per query that probes it. Here the
// (query, probe) pairs of a chunk of probe ranks are grouped by list: an item is
// one list and up to 64 of the queries that probe it, so the list's codes are
// read and unpacked once for the whole group. The integer inner products
// ip = sum_d b01_d qu_d of 16 vectors x 16 queries are one
// v_mfma_i32_16x16x64_i8 per 64 dimensions (codes unpacked to 0/1 bytes as the
// A operand, the queries' quantised residuals as the B operand), then the same
// estimator epilogue as the popcount scan (Eqs. rabitq-ip-estimator,
// approx-dist) gives bit-identical d_hat^2. Candidates at or below the query's
// threshold (its exact R-th estimate after the previous chunk) are appended to
// the query's pool; the pass of a query whose pool would overflow is redone by
// the query-major scan. Items come from a persistent work queue
// (Sec. 3.3.1: work is balanced over index blocks, not over queries).
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "kernels.hpp"

namespace rbq {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int GMAX = 64;   // queries per item (four 16-query MFMA tiles)
constexpr int KSMAX = 4;   // 64-dimension MFMA steps (D <= 256)
constexpr int STAGE = 512; // survivors staged per wave before a flush

// ---- inverted map of the chunk's pairs: list -> pairs probing it ----------

__global__ void k_grp_hist(const int32_t* __restrict__ probes, int nq, int nprobe, int p0, int pn,
                           int32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nq * pn) return;
  const int64_t i = t / pn;
  const int p = p0 + (int)(t - i * pn);
  const int j = probes[i * nprobe + p];
  if (j >= 0) atomicAdd(&cnt[j], 1);  // (-1: the query probes fewer lists)
}

// Exclusive prefix sums over lists of the pair counts and of the item counts
// ceil(cnt / G); one workgroup; also clears the scatter cursors.
__global__ __launch_bounds__(256) void k_grp_offsets(const int32_t* __restrict__ cnt, int nlist,
                                                     int G, int32_t* __restrict__ pair_off,
                                                     int32_t* __restrict__ item_off,
                                                     int32_t* __restrict__ fill) {
  __shared__ int32_t sp[256], si[256];
  const int tid = threadIdx.x;
  const int per = (nlist + 255) / 256;
  const int j0 = tid * per, j1 = min(nlist, j0 + per);
  int32_t ps = 0, is = 0;
  for (int j = j0; j < j1; ++j) {
    ps += cnt[j];
    is += (cnt[j] + G - 1) / G;
  }
  sp[tid] = ps;
  si[tid] = is;
  __syncthreads();
  if (tid == 0) {
    int32_t a = 0, b = 0;
    for (int t = 0; t < 256; ++t) {
      const int32_t x = sp[t], y = si[t];
      sp[t] = a;
      si[t] = b;
      a += x;
      b += y;
    }
    pair_off[nlist] = a;
    item_off[nlist] = b;
  }
  __syncthreads();
  int32_t a = sp[tid], b = si[tid];
  for (int j = j0; j < j1; ++j) {
    pair_off[j] = a;
    item_off[j] = b;
    a += cnt[j];
    b += (cnt[j] + G - 1) / G;
    fill[j] = 0;
  }
}

// One descriptor per item: (list, first slot of its pairs, number of pairs).
__global__ void k_grp_items(const int32_t* __restrict__ cnt, const int32_t* __restrict__ pair_off,
                            const int32_t* __restrict__ item_off, int nlist, int G,
                            int4* __restrict__ items) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlist) return;
  const int c = cnt[j];
  for (int g = 0; g * G < c; ++g)
    items[item_off[j] + g] = make_int4(j, pair_off[j] + g * G, min(G, c - g * G), 0);
}

__global__ void k_grp_scatter(const int32_t* __restrict__ probes, int nq, int nprobe, int p0, int pn,
                              const int32_t* __restrict__ pair_off, int32_t* __restrict__ fill,
                              int32_t* __restrict__ slots) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nq * pn) return;
  const int64_t i = t / pn;
  const int p = p0 + (int)(t - i * pn);
  const int64_t pair = i * nprobe + p;
  const int j = probes[pair];
  if (j >= 0) slots[pair_off[j] + atomicAdd(&fill[j], 1)] = (int32_t)pair;
}

__device__ inline uint32_t lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// 16 code bits -> 16 bytes of 0/1 (byte b = bit b), as four dwords.
__device__ inline v4i unpack16(uint32_t bits) {
  v4i r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = (int)((((bits >> (4 * q)) & 0xFu) * 0x00204081u) & 0x01010101u);
  return r;
}

template <int KS>
__global__ __launch_bounds__(256) void k_scan_group(GroupArgs a) {
  __shared__ v4i sB[GMAX / 16][KS][64];      // B operands: [query tile][k step][lane]
  __shared__ float4 sSc[GMAX];                // (||r||^2, v_l, Delta, sum qu) per query slot
  __shared__ float sThr[GMAX];                // threshold on d_hat^2 per query slot
  __shared__ int32_t sQ[GMAX];                // query id per slot
  __shared__ uint32_t sCode[4][2 * KS][64];  // per wave: the micro-block's code words
  __shared__ __align__(16) float sVx[4][64], sAdd[4][64], sMul[4][64];
  // per wave: survivors as (float bits of d_hat^2 << 32) | (query slot << 26 |
  // position in the list)
  __shared__ uint64_t sStage[4][STAGE];
  __shared__ uint32_t sFcnt[4][GMAX], sFbase[4][GMAX];  // per wave: flush counts and bases
  __shared__ int32_t sItem;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int W = a.L.W;
  const int D = a.L.d;
  const int Wq = W * 32;  // qu bytes per pair
  const int nlist = a.nlist;
  int stage_n = 0;  // wave-uniform fill of this wave's stage
  // Moves the staged survivors to their queries' pools: the entries are
  // counted per query slot in LDS, each slot reserves its range with one
  // global atomic, and every entry is written at its slot's base plus its
  // rank (ids looked up lane-parallel).
  int list_pos0 = 0;  // first position of the item's list
  auto flush = [&](int nst) {
    if (nst == 0) return;
    sFcnt[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) atomicAdd(&sFcnt[wave][(uint32_t)sStage[wave][e] >> 26], 1u);
    __builtin_amdgcn_wave_barrier();
    const uint32_t c = sFcnt[wave][lane];
    sFbase[wave][lane] = c ? atomicAdd(&a.pcnt[sQ[lane]], c) : 0u;
    sFcnt[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) {
      const uint64_t kp = sStage[wave][e];
      const uint32_t lo = (uint32_t)kp;
      const int q = (int)(lo >> 26);
      const int qi = sQ[q];
      const uint32_t slot = sFbase[wave][q] + atomicAdd(&sFcnt[wave][q], 1u);
      const int id = a.L.pos2id[list_pos0 + (int)(lo & 0x3FFFFFFu)];
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
  const int total = a.item_off[nlist];
  for (;;) {
    if (tid == 0) sItem = (int32_t)atomicAdd(a.item_counter, 1u);
    __syncthreads();
    const int item = sItem;
    __syncthreads();  // sItem is rewritten at the next item
    if (item >= total) break;
    const int4 it = a.items[item];
    const int j = it.x, first = it.y, count = it.z;
    const int nt = (count + 15) >> 4;
    // stage the group's queries
    if (tid < GMAX) {
      if (tid < count) {
        const int pair = a.slots[first + tid];
        const int qi = pair / a.nprobe;
        sQ[tid] = qi;
        sSc[tid] = a.scal[pair];
        const uint32_t th = a.qthr[qi];
        sThr[tid] = th == 0xFFFFFFFFu ? INFINITY : f32_ord(th);
      } else {
        sQ[tid] = -1;
      }
    }
    for (int e = tid; e < (GMAX / 16) * KS * 64; e += 256) {
      const int n = e / (KS * 64), t = (e / 64) % KS, l = e & 63;
      const int q = 16 * n + (l & 15);
      const int off = 64 * t + 16 * (l >> 4);
      v4i v = {0, 0, 0, 0};
      if (q < count && off < Wq) {
        const int pair = a.slots[first + q];
        v = *reinterpret_cast<const v4i*>(a.qu + (int64_t)pair * Wq + off);
      }
      sB[n][t][l] = v;
    }
    __syncthreads();
    // this lane's query (column lane & 15 of each 16-query tile): scalars in
    // registers for the whole item; an empty slot gets a NaN threshold
    float qrn2[GMAX / 16], qvl[GMAX / 16], qdelta[GMAX / 16], qthr[GMAX / 16];
    int qsum[GMAX / 16];
#pragma unroll
    for (int n = 0; n < GMAX / 16; ++n) {
      const int q = 16 * n + (lane & 15);
      const float4 sc = sSc[q];
      qrn2[n] = sc.x;
      qvl[n] = sc.y;
      qdelta[n] = sc.z;
      qsum[n] = -(int)sc.w;  // negated: the estimate adds it
      qthr[n] = q < count ? sThr[q] : NAN;
    }
    const int len = a.L.list_len[j], mb0 = a.L.list_mb[j];
    const int nmb = (len + 63) >> 6;
    list_pos0 = mb0 << 6;
    const size_t rec = (size_t)(W + 2) * 64;
    // lane = vector of the micro-block; the next micro-block's words and
    // factors are loaded into registers while the current one is computed
    uint32_t cw[2 * KS];
    float fa = 0.f, fm = 0.f;
    auto load_mb = [&](int mbi) {
      const uint32_t* blk = a.L.blocks + (size_t)(mb0 + mbi) * rec;
#pragma unroll
      for (int w = 0; w < 2 * KS; ++w) cw[w] = w < W ? blk[w * 64 + lane] : 0u;
      fa = __uint_as_float(blk[W * 64 + lane]);
      fm = __uint_as_float(blk[(W + 1) * 64 + lane]);
    };
    if (wave < nmb) load_mb(wave);
    for (int mb = wave; mb < nmb; mb += 4) {
      {
        int pop = 0;
#pragma unroll
        for (int w = 0; w < 2 * KS; ++w) {
          sCode[wave][w][lane] = cw[w];
          pop += __popc(cw[w]);
        }
        sVx[wave][lane] = rbq_vx(fm, pop, D);
        const bool valid = (mb << 6) + lane < len;
        sAdd[wave][lane] = valid ? fa : NAN;
        sMul[wave][lane] = fm;
      }
      __builtin_amdgcn_wave_barrier();
      if (mb + 4 < nmb) load_mb(mb + 4);
      const int lg = lane >> 4;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        v4i A[KS];
        const int vrow = 16 * m + (lane & 15);
#pragma unroll
        for (int t = 0; t < KS; ++t) {
          const uint32_t word = sCode[wave][2 * t + (lg >> 1)][vrow];
          A[t] = unpack16((word >> (16 * (lg & 1))) & 0xFFFFu);
        }
        // the four vectors of this lane's result rows: 16 m + 4 lg + r
        const float4 fadd4 = *reinterpret_cast<const float4*>(&sAdd[wave][16 * m + 4 * lg]);
        const float4 vx4 = *reinterpret_cast<const float4*>(&sVx[wave][16 * m + 4 * lg]);
        const float4 fmul4 = *reinterpret_cast<const float4*>(&sMul[wave][16 * m + 4 * lg]);
        const float fadd[4] = {fadd4.x, fadd4.y, fadd4.z, fadd4.w};
        const float vxr[4] = {vx4.x, vx4.y, vx4.z, vx4.w};
        const float fmul[4] = {fmul4.x, fmul4.y, fmul4.z, fmul4.w};
        // position in the list of this lane's first result row
        const uint32_t rel0 = (uint32_t)((mb << 6) + 16 * m + 4 * lg);
#pragma unroll
        for (int n = 0; n < GMAX / 16; ++n) {
          if (n >= nt) break;
          v4i acc = {0, 0, 0, 0};
#pragma unroll
          for (int t = 0; t < KS; ++t)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[t], sB[n][t][lane], acc, 0, 0, 0);
          float est[4];
          bool pass[4];
          bool anyp = false;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            est[r] = rbq_estimate(qrn2[n], qvl[n], qdelta[n], qsum[n], acc[r], fadd[r], fmul[r], vxr[r]);
            pass[r] = est[r] <= qthr[n];  // NaN (padding lanes, empty slots) never passes
            anyp |= pass[r];
          }
          if (__ballot(anyp)) {  // stage the survivors of this tile
            const uint32_t tag = rel0 | ((uint32_t)(16 * n + (lane & 15)) << 26);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const uint64_t mask = __ballot(pass[r]);
              if (pass[r]) {
                const int e = stage_n + (int)lane_prefix(mask);
                sStage[wave][e] = ((uint64_t)__float_as_uint(est[r]) << 32) | (tag + (uint32_t)r);
              }
              stage_n += (int)__popcll(mask);
            }
            if (stage_n > STAGE - 256) {
              __builtin_amdgcn_wave_barrier();
              flush(stage_n);
              stage_n = 0;
            }
          }
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    __builtin_amdgcn_wave_barrier();
    flush(stage_n);
    stage_n = 0;
    __syncthreads();  // the group's LDS is restaged for the next item
  }
}

void launch_group_map(hipStream_t s, const int32_t* probes, int nq, int nprobe, int p0, int pn,
                      int nlist, int G, int32_t* cnt, int32_t* pair_off, int32_t* item_off,
                      int32_t* fill, int32_t* slots, int4* items) {
  const int64_t pairs = (int64_t)nq * pn;
  RBQ_HIP(hipMemsetAsync(cnt, 0, nlist * sizeof(int32_t), s));
  hipLaunchKernelGGL(k_grp_hist, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, probes, nq,
                     nprobe, p0, pn, cnt);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grp_offsets, dim3(1), dim3(256), 0, s, cnt, nlist, G, pair_off, item_off, fill);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grp_items, dim3((nlist + 255) / 256), dim3(256), 0, s, cnt, pair_off, item_off,
                     nlist, G, items);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grp_scatter, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, probes,
                     nq, nprobe, p0, pn, pair_off, fill, slots);
  RBQ_HIP(hipGetLastError());
}

int group_k_steps(int d) { return (d + 63) / 64; }

void launch_scan_group(hipStream_t s, const GroupArgs& a, int workgroups) {
  RBQ_CHECK(a.G >= 1 && a.G <= GMAX, "group size out of range");
  const int ks = group_k_steps(a.L.d);
  RBQ_CHECK(ks <= KSMAX, "grouped scan supports d <= 256");
  switch (ks) {
    case 1: hipLaunchKernelGGL(k_scan_group<1>, dim3(workgroups), dim3(256), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_scan_group<2>, dim3(workgroups), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_scan_group<3>, dim3(workgroups), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL(k_scan_group<4>, dim3(workgroups), dim3(256), 0, s, a); break;
  }
  RBQ_HIP(hipGetLastError());
}

// Queries whose pool overflowed in a list-major pass are searched again from
// scratch by the query-major scan: empty running top-R, no threshold, empty
// pool.
__global__ void k_reset_masked(const uint32_t* __restrict__ mask, uint64_t* __restrict__ rows, int64_t ld,
                               int R, uint32_t* __restrict__ qthr, uint32_t* __restrict__ pcnt) {
  const int64_t i = blockIdx.x;
  if (!mask[i]) return;
  for (int c = threadIdx.x; c < R; c += blockDim.x) rows[i * ld + c] = KEY_NONE;
  if (threadIdx.x == 0) {
    qthr[i] = 0xFFFFFFFFu;
    pcnt[i] = 0u;
  }
}

void launch_reset_masked(hipStream_t s, const uint32_t* mask, uint64_t* rows, int64_t ld, int R,
                         uint32_t* qthr, uint32_t* pcnt, int nq) {
  if (nq <= 0) return;
  hipLaunchKernelGGL(k_reset_masked, dim3(nq), dim3(256), 0, s, mask, rows, ld, R, qthr, pcnt);
  RBQ_HIP(hipGetLastError());
}

}  // namespace rbq
