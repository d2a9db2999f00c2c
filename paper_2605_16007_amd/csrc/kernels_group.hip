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
constexpr int STAGE = 512; // candidates staged per wave before a flush

// ---- inverted map of the list-major chunks' pairs: list -> pairs ----------
// Built once per search for all list-major chunks (a suffix of the probe
// ranks): bin c * nlist + j holds the pairs of chunk c that probe list j. The
// work grows with the pairs, not with nlist x nq:
//   count: each pair adds one to its bin (atomic);
//   sums:  each workgroup of 16 lists adds up its bins' pairs and items per
//          chunk, an item being one index block of the list (B micro-blocks;
//          B = 0: the whole list) and up to G of its pairs;
//   scan:  one workgroup turns the workgroup sums (chunk-major) into bases,
//          and the item range of every chunk;
//   bins:  one wave per bin finds its pair and item bases and writes its
//          items, block-major (the query groups of one block are consecutive
//          items, so they run close together and share its reads);
//   fill:  each pair takes the next slot of its bin (atomic). The order of
//          the pairs inside a bin is not fixed, and nothing depends on it: a
//          scan's survivors are merged by an exact selection.

constexpr int kMapLists = 16;  // lists per workgroup of the map's sums

// chunk of list-major probe rank p (-1 for no pair): bounds are ascending
__device__ inline int map_chunk(const GroupChunks& gc, int p) {
  int ch = p >= 0 ? 0 : -1;
#pragma unroll
  for (int b = 1; b < kMaxGroupChunks; ++b) {
    if (b >= gc.nb) continue;  // (the bound is uniform: every later b too)
    ch += p >= gc.bound[b] ? 1 : 0;
  }
  return ch;
}

__device__ inline int32_t wave_sum(int32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ inline uint32_t lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

// index blocks of a list of `len` vectors (B micro-blocks each; 0: one block)
__device__ inline int map_blocks(int len, int B) {
  return B > 0 ? max(1, (((len + 63) >> 6) + B - 1) / B) : 1;
}

// (x: 256 probe ranks per workgroup from the first list-major rank; y:
// queries, striding by gridDim.y)
template <bool FILL>
__global__ void k_map_pairs(const int32_t* __restrict__ probes, int nq, int nprobe, GroupChunks gc,
                            int nlist, int32_t* __restrict__ cnt, const int32_t* __restrict__ bbase,
                            int32_t* __restrict__ fillc, int32_t* __restrict__ slots) {
  const int p = gc.bound[0] + (int)blockIdx.x * 256 + (int)threadIdx.x;
  if (p >= nprobe) return;
  const int c = map_chunk(gc, p);
  for (int64_t i = blockIdx.y; i < nq; i += gridDim.y) {
    const int64_t pair = i * nprobe + p;
    const int j = probes[pair];
    if (j < 0) continue;
    const int64_t bin = (int64_t)c * nlist + j;
    if (FILL)
      slots[bbase[bin] + atomicAdd(&fillc[bin], 1)] = (int32_t)pair;
    else
      atomicAdd(&cnt[bin], 1);
  }
}

// per (chunk, workgroup of 16 lists): pairs and items (one wave, grid (nwg, nb))
__global__ void k_map_sums(const int32_t* __restrict__ cnt, const int32_t* __restrict__ list_len, int nlist,
                           int G, int B, int nwg, int nb, int32_t* __restrict__ wpart) {
  const int wg = blockIdx.x, c = blockIdx.y, lane = threadIdx.x;
  const int j = wg * kMapLists + lane;
  int32_t pc = 0, ic = 0;
  if (lane < kMapLists && j < nlist) {
    pc = cnt[(int64_t)c * nlist + j];
    ic = ((pc + G - 1) / G) * map_blocks(list_len[j], B);
  }
  pc = wave_sum(pc);
  ic = wave_sum(ic);
  if (lane == 0) {
    wpart[c * nwg + wg] = pc;
    wpart[(nb + c) * nwg + wg] = ic;
  }
}

// In place: wpart[0..V) pair sums and wpart[V..2V) item sums (V = nb * nwg,
// chunk-major) become exclusive bases; chunk_items[c] = the first item of
// chunk c (chunk_items[nb] = all items). One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_grp_scan(int32_t* __restrict__ wpart, int V, int nwg, int nb,
                                                   int32_t* __restrict__ chunk_items) {
  __shared__ int32_t wp[16], wi[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int32_t carry_p = 0, carry_i = 0;
  for (int v0 = 0; v0 < V; v0 += 1024) {
    const int v = v0 + tid;
    const int32_t p = v < V ? wpart[v] : 0, it = v < V ? wpart[V + v] : 0;
    int32_t xp = p, xi = it;
    for (int off = 1; off < 64; off <<= 1) {
      const int32_t tp = __shfl_up(xp, off), ti = __shfl_up(xi, off);
      if (lane >= off) {
        xp += tp;
        xi += ti;
      }
    }
    if (lane == 63) {
      wp[wave] = xp;
      wi[wave] = xi;
    }
    __syncthreads();
    int32_t a = carry_p + xp - p, bi = carry_i + xi - it;
#pragma unroll
    for (int w = 0; w < 16; ++w) {
      const int32_t tp = wp[w], ti = wi[w];
      if (w < wave) {
        a += tp;
        bi += ti;
      }
      carry_p += tp;
      carry_i += ti;
    }
    __syncthreads();
    if (v < V) {
      wpart[v] = a;
      wpart[V + v] = bi;
      if (v % nwg == 0) chunk_items[v / nwg] = bi;
    }
  }
  if (tid == 0) chunk_items[nb] = carry_i;
}

// one wave per bin (c, j): its pair base (kept for the fill) and its items
__global__ void k_map_bins(const int32_t* __restrict__ cnt, const int32_t* __restrict__ list_mb,
                           const int32_t* __restrict__ list_len, int nlist, int G, int B, int nwg, int nb,
                           const int32_t* __restrict__ wpart, int32_t* __restrict__ bbase,
                           int4* __restrict__ items) {
  const int64_t bin = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (bin >= (int64_t)nb * nlist) return;
  const int c = (int)(bin / nlist), j = (int)(bin - (int64_t)c * nlist);
  const int wg = j / kMapLists, j0 = wg * kMapLists;
  // the lists of this workgroup before j
  int32_t pc = 0, ic = 0;
  if (lane < j - j0) {
    const int jl = j0 + lane;
    pc = cnt[(int64_t)c * nlist + jl];
    ic = ((pc + G - 1) / G) * map_blocks(list_len[jl], B);
  }
  const int32_t pb = wpart[c * nwg + wg] + wave_sum(pc);
  const int32_t ib = wpart[(nb + c) * nwg + wg] + wave_sum(ic);
  const int32_t cn = cnt[bin];
  if (lane == 0) bbase[bin] = pb;
  if (cn == 0) return;
  const int len = list_len[j], mb = list_mb[j];
  const int nblk = map_blocks(len, B), ng = (cn + G - 1) / G;
  const int bl = B > 0 ? B * 64 : len;  // vectors per block
  for (int t = lane; t < nblk * ng; t += 64) {
    const int blk = t / ng, g = t - blk * ng;
    items[ib + t] = make_int4(mb + (B > 0 ? blk * B : 0), pb + g * G, min(G, cn - g * G),
                              min(bl, len - blk * bl));
  }
}

// 16 code bits -> 16 bytes of 0/1 (byte b = bit b), as four dwords.
__device__ inline v4i unpack16(uint32_t bits) {
  v4i r;
#pragma unroll
  for (int q = 0; q < 4; ++q) r[q] = (int)((((bits >> (4 * q)) & 0xFu) * 0x00204081u) & 0x01010101u);
  return r;
}

// The MFMA multiplies signed bytes. QB (query bytes) says how qu becomes the
// B operand:
//   QB_DOUBLE (B_q <= 6): B = 2 qu <= 126 and the accumulator starts at
//     -sum qu, so the MFMA returns g = 2 ip - sum qu itself;
//   QB_PLAIN (B_q = 7): B = qu <= 127, g = (ip << 1) - sum qu;
//   QB_OFFSET (B_q = 8): B = qu - 128 and the accumulator starts at 128 pop
//     (pop = the vector's popcount), so the MFMA still returns ip.
// GT: 16-query tiles per item (G <= 16 GT); each lane keeps its B operands
// for the whole item in registers.
//   QB_F8 (B_q <= 4): the codes as fp4 (E2M1, 1.0 per set bit) and B = 2 qu
//     as fp8 (E4M3; 2 qu <= 30 is exact), accumulated in fp32 from -sum qu:
//     g comes out as an exactly integral float and no conversion is needed.
//     Each step covers 128 dimensions (KS counts these steps); lane group g
//     of a row expands code word g of the step by shifts and masks (bit
//     4 i + q -> nibble i of dword q), and the quantiser writes the pair's
//     B bytes in the matching order, so staging B is a plain 32-byte load.
enum { QB_DOUBLE = 0, QB_PLAIN = 1, QB_OFFSET = 2, QB_F8 = 3 };
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));
// DUMP (debug entry point only): every estimate of the item is also written
// out per (pair, position in the list) with its inner product ip, before any
// threshold test.
template <int KS, int QB, int GT, bool DUMP>
__global__ __launch_bounds__(256) void k_scan_group(GroupArgs a) {
  constexpr bool F8 = QB == QB_F8;
  constexpr int CW = F8 ? 4 * KS : 2 * KS;  // code words per vector staged
  using BT = typename std::conditional<F8, v8i, v4i>::type;
  using AccT = typename std::conditional<F8, v4f, v4i>::type;
  __shared__ BT sB[GT][KS][64];              // B operands: [query tile][k step][lane]
  __shared__ float4 sSc[GMAX];                // (||r||^2, v_l, Delta, sum qu) per query slot
  __shared__ float sThr[GMAX];                // threshold on d_hat^2 per query slot
  __shared__ int32_t sQ[GMAX];                // query id per slot
  __shared__ int32_t sPair[DUMP ? GMAX : 1];  // (query, probe) pair per slot
  __shared__ uint32_t sCode[4][CW][64];      // per wave: the micro-block's code words
  __shared__ __align__(16) float sVx[4][64], sAdd[4][64], sMul[4][64];
  __shared__ __align__(16) int32_t sPop[QB == QB_OFFSET ? 4 : 1][64];  // 128 pop per vector
  // per wave: candidates that passed the scan's test, as (float bits of the
  // tested value << 32) | (query slot << 26 | position in the list)
  __shared__ uint64_t sStage[4][STAGE];
  __shared__ uint32_t sFcnt[4][GMAX], sFbase[4][GMAX];  // per wave: flush counts and bases
  __shared__ int32_t sItem;
  // 8 code bits -> 8 bytes of 0/1 (byte b = bit b): the unpacking of the A
  // operand is two table reads per 16 bits
  __shared__ uint2 sLut[F8 ? 1 : 256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int W = a.L.W;
  const int D = a.L.d;
  const int Wq = W * 32;  // qu bytes per pair
  int stage_n = 0;  // wave-uniform fill of this wave's stage
  // Moves the staged candidates to their queries' pools. First each entry
  // forms d_hat^2 (QB_F8 staged the value without ||r||^2) and takes the
  // exact test against its query's threshold; the passing entries are counted
  // per query slot in LDS, each slot reserves its range with one global
  // atomic, and every entry is written at its slot's base plus its rank (ids
  // looked up lane-parallel).
  int list_pos0 = 0;  // first position of the item's list
  auto flush = [&](int nst) {
    sFcnt[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) {
      const uint64_t kp = sStage[wave][e];
      const uint32_t lo = (uint32_t)kp;
      const int q = (int)(lo >> 26);
      const float v = __uint_as_float((uint32_t)(kp >> 32));
      const float est = F8 ? v + sSc[q].x : v;  // d_hat^2, as every scan forms it
      if (est <= sThr[q]) {
        atomicAdd(&sFcnt[wave][q], 1u);
        sStage[wave][e] = ((uint64_t)__float_as_uint(est) << 32) | lo;
      } else {
        sStage[wave][e] = ~0ull;
      }
    }
    __builtin_amdgcn_wave_barrier();
    const uint32_t c = sFcnt[wave][lane];
    sFbase[wave][lane] = c ? atomicAdd(&a.pcnt[sQ[lane]], c) : 0u;
    sFcnt[wave][lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    for (int e = lane; e < nst; e += 64) {
      const uint64_t kp = sStage[wave][e];
      if (kp != ~0ull) {
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
    }
    __builtin_amdgcn_wave_barrier();
  };
  const int first_item = a.item_off[0], end_item = a.item_off[1];
  if (!F8 && tid < 256) {
    const v4i u = unpack16((uint32_t)tid);
    sLut[tid] = make_uint2((uint32_t)u[0], (uint32_t)u[1]);
  }
  // (the first item's barriers order these writes before any read)
  for (;;) {
    if (tid == 0) sItem = first_item + (int32_t)atomicAdd(a.item_counter, 1u);
    __syncthreads();
    const int item = sItem;
    __syncthreads();  // sItem is rewritten at the next item
    if (item >= end_item) break;
    const int4 it = a.items[item];
    const int first = it.y, count = it.z;
    const int nt = (count + 15) >> 4;
    const int mb0 = it.x, len = it.w;
    const int nmb = (len + 63) >> 6;
    list_pos0 = mb0 << 6;
    // (debug dumps: the item's index block starts this many vectors into its list)
    const int blk_off = DUMP ? list_pos0 - (a.L.list_mb[a.probes[a.slots[first]]] << 6) : 0;
    const size_t rec = (size_t)(W + 2) * 64;
    // lane = vector of the micro-block; the next micro-block's words and
    // factors are loaded into registers while the current one is computed
    // (the first ones are in flight while the item's queries are staged)
    uint32_t cw[CW];
    float fa = 0.f, fm = 0.f;
    auto load_mb = [&](int mbi) {
      const uint32_t* blk = a.L.blocks + (size_t)(mb0 + mbi) * rec;
#pragma unroll
      for (int w = 0; w < CW; ++w) cw[w] = w < W ? blk[w * 64 + lane] : 0u;
      fa = __uint_as_float(blk[W * 64 + lane]);
      fm = __uint_as_float(blk[(W + 1) * 64 + lane]);
    };
    if (wave < nmb) load_mb(wave);
    // stage the group's queries
    if (tid < GMAX) {
      if (tid < count) {
        const int pair = a.slots[first + tid];
        const int qi = pair / a.nprobe;
        sQ[tid] = qi;
        if (DUMP) sPair[tid] = pair;
        sSc[tid] = a.scal[pair];
        const uint32_t th = a.qthr[qi];
        sThr[tid] = th == 0xFFFFFFFFu ? INFINITY : f32_ord(th);
      } else {
        sQ[tid] = -1;
      }
    }
    for (int e = tid; e < GT * KS * 64; e += 256) {
      const int n = e / (KS * 64), t = (e / 64) % KS, l = e & 63;
      const int q = 16 * n + (l & 15);
      const int off = 64 * t + 16 * (l >> 4);
      BT v = {};
      if constexpr (F8) {
        if (q < count) {
          const int pair = a.slots[first + q];
          v = *reinterpret_cast<const v8i*>(a.qu + (int64_t)pair * a.qu_ld + 128 * t + 32 * (l >> 4));
        }
      } else {
        if (q < count && off < Wq) {
          const int pair = a.slots[first + q];
          v = *reinterpret_cast<const v4i*>(a.qu + (int64_t)pair * a.qu_ld + off);
          if (QB == QB_DOUBLE) v <<= 1;  // bytes <= 63: no carry into the next byte
          if (QB == QB_OFFSET) v ^= (int)0x80808080u;  // qu - 128 as a signed byte
        }
      }
      sB[n][t][l] = v;
    }
    __syncthreads();
    // this lane's query (column lane & 15 of each 16-query tile): its B
    // operands and scalars in registers for the whole item; an empty slot
    // gets a NaN threshold
    BT Bq[GT][KS];
    float qrn2[GT], qvl[GT], qdelta[GT], qthr[GT], qbound[GT];
    int qneg[GT];
#pragma unroll
    for (int n = 0; n < GT; ++n) {
      const int q = 16 * n + (lane & 15);
      const float4 sc = sSc[q];
      qrn2[n] = sc.x;
      qvl[n] = sc.y;
      qdelta[n] = sc.z;
      qneg[n] = -(int)sc.w;
      qthr[n] = q < count ? sThr[q] : NAN;
      if (F8) qbound[n] = rbq_part_bound(qthr[n], qrn2[n]);
#pragma unroll
      for (int t = 0; t < KS; ++t) Bq[n][t] = sB[n][t][lane];
    }
    for (int mb = wave; mb < nmb; mb += 4) {
      {
        int pop = 0;
#pragma unroll
        for (int w = 0; w < CW; ++w) {
          sCode[wave][w][lane] = cw[w];
          pop += __popc(cw[w]);
        }
        sVx[wave][lane] = rbq_vx(fm, pop, D);
        if (QB == QB_OFFSET) sPop[wave][lane] = pop << 7;
        const bool valid = (mb << 6) + lane < len;
        sAdd[wave][lane] = valid ? fa : NAN;
        sMul[wave][lane] = fm;
      }
      __builtin_amdgcn_wave_barrier();
      if (mb + 4 < nmb) load_mb(mb + 4);
      const int lg = lane >> 4;
      // A operands of row block m (vectors 16 m + (lane & 15)). For small
      // items those of block m + 1 are read from LDS before block m's
      // epilogue, so the reads are in flight while it computes (for larger
      // items the extra registers would cost a wave of occupancy)
      constexpr bool pre = F8 ? KS * GT <= 2 : KS * GT <= 4;
      auto unpack_a = [&](int m, v4i (&A)[KS]) __attribute__((always_inline)) {
        const int vrow = 16 * m + (lane & 15);
#pragma unroll
        for (int t = 0; t < KS; ++t) {
          if constexpr (F8) {
            const uint32_t w = sCode[wave][4 * t + lg][vrow];
            A[t] = v4i{(int)((w << 1) & 0x22222222u), (int)(w & 0x22222222u), (int)((w >> 1) & 0x22222222u),
                       (int)((w >> 2) & 0x22222222u)};
          } else {
            const uint32_t word = sCode[wave][2 * t + (lg >> 1)][vrow];
            const uint2 lo8 = sLut[(word >> (16 * (lg & 1))) & 0xFFu];
            const uint2 hi8 = sLut[(word >> (16 * (lg & 1) + 8)) & 0xFFu];
            A[t] = v4i{(int)lo8.x, (int)lo8.y, (int)hi8.x, (int)hi8.y};
          }
        }
      };
      v4i An[KS];
      unpack_a(0, An);
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        v4i A[KS];
        if (pre || m == 0) {
#pragma unroll
          for (int t = 0; t < KS; ++t) A[t] = An[t];
        } else {
          unpack_a(m, A);
        }
        // every query tile's products first, then the epilogues
        v4i c0 = {0, 0, 0, 0};
        if (QB == QB_OFFSET) c0 = *reinterpret_cast<const v4i*>(&sPop[QB == QB_OFFSET ? wave : 0][16 * m + 4 * lg]);
        AccT acc[GT];
#pragma unroll
        for (int n = 0; n < GT; ++n) {
          if (n < nt) {
            // QB_DOUBLE: the accumulator starts at -sum qu, so it ends at g
            if constexpr (F8) {
              const float qf = (float)qneg[n];
              v4f c = {qf, qf, qf, qf};
#pragma unroll
              for (int t = 0; t < KS; ++t) {
                const v8i a8 = {A[t][0], A[t][1], A[t][2], A[t][3], 0, 0, 0, 0};
                // A fp4 (format 4), B fp8 E4M3 (format 0), unit scales
                c = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a8, Bq[n][t], c, 4, 0, 0, 0, 0, 0);
              }
              acc[n] = c;
            } else {
              v4i c = QB == QB_DOUBLE ? v4i{qneg[n], qneg[n], qneg[n], qneg[n]} : c0;
#pragma unroll
              for (int t = 0; t < KS; ++t) c = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[t], Bq[n][t], c, 0, 0, 0);
              acc[n] = c;
            }
          }
        }
        if (pre && m < 3) unpack_a(m + 1, An);
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
        for (int n = 0; n < GT; ++n) {
          if (n >= nt) break;
          // QB_F8: the estimate without ||r||^2 is tested against the
          // query's bound on it; the lanes that pass are staged, and the
          // flush forms the estimate and tests it exactly
          float part[4];
          bool ok[4];      // this lane's value may pass, per result row
          uint64_t pm[4];  // the lanes that may pass, per result row
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if constexpr (F8) {
              part[r] = rbq_estimate_part(qvl[n], qdelta[n], acc[n][r], fadd[r], fmul[r], vxr[r]);
              // NaN (padding lanes, empty slots) never passes
              ok[r] = part[r] <= qbound[n];
            } else {  // (the signed-byte forms test the estimate itself: fewer registers)
              const int g = QB == QB_DOUBLE ? acc[n][r] : (acc[n][r] << 1) + qneg[n];
              part[r] = rbq_estimate_g(qrn2[n], qvl[n], qdelta[n], g, fadd[r], fmul[r], vxr[r]);
              ok[r] = part[r] <= qthr[n];
            }
            pm[r] = __builtin_amdgcn_ballot_w64(ok[r]);
            if constexpr (DUMP) {
              const int q = 16 * n + (lane & 15);
              const uint32_t pos = rel0 + (uint32_t)r;
              if (q < count && pos < (uint32_t)len) {
                // g = 2 ip - sum qu (QB_F8, QB_DOUBLE) or ip itself
                const int sq = -qneg[n];
                int ip;
                if constexpr (F8)
                  ip = ((int)acc[n][r] + sq) >> 1;
                else if constexpr (QB == QB_DOUBLE)
                  ip = (acc[n][r] + sq) >> 1;
                else
                  ip = acc[n][r];
                const int64_t o = (int64_t)sPair[q] * a.maxlen + blk_off + pos;
                a.dump_ip[o] = ip;
                a.dump_est[o] = F8 ? part[r] + qrn2[n] : part[r];
              }
            }
          }
          if (pm[0] | pm[1] | pm[2] | pm[3]) {  // stage this tile's candidates
            const uint32_t tag = rel0 | ((uint32_t)(16 * n + (lane & 15)) << 26);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (pm[r]) {
                if (ok[r]) {
                  const uint32_t e = __builtin_amdgcn_mbcnt_hi(
                      (uint32_t)(pm[r] >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)pm[r], (uint32_t)stage_n));
                  sStage[wave][e] = ((uint64_t)__float_as_uint(part[r]) << 32) | (tag + (uint32_t)r);
                }
                stage_n += (int)__popcll(pm[r]);
              }
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

void launch_group_map(hipStream_t s, const int32_t* probes, int nq, int nprobe, const GroupChunks& gc,
                      int nlist, int G, int B, const int32_t* list_mb, const int32_t* list_len,
                      const GroupMap& m) {
  RBQ_CHECK(gc.nb >= 1 && gc.nb <= kMaxGroupChunks && gc.bound[gc.nb] == nprobe,
            "list-major chunk bounds");
  RBQ_CHECK(G >= 1 && B >= 0, "list-major map: item shape");
  const int64_t pairs = (int64_t)nq * (nprobe - gc.bound[0]);
  if (pairs <= 0) return;
  const int nwg = group_map_workgroups(nlist);
  const int span = nprobe - gc.bound[0];
  const dim3 pg((unsigned)((span + 255) / 256), (unsigned)std::min(nq, 65535));
  // (cnt and fill are zero: the search's state initialisation clears them)
  hipLaunchKernelGGL(k_map_pairs<false>, pg, dim3(256), 0, s, probes, nq, nprobe, gc, nlist, m.cnt, nullptr,
                     nullptr, nullptr);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_map_sums, dim3(nwg, gc.nb), dim3(64), 0, s, m.cnt, list_len, nlist, G, B, nwg, gc.nb,
                     m.wpart);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_grp_scan, dim3(1), dim3(1024), 0, s, m.wpart, gc.nb * nwg, nwg, gc.nb, m.chunk_items);
  RBQ_HIP(hipGetLastError());
  const int64_t bins = (int64_t)gc.nb * nlist;
  hipLaunchKernelGGL(k_map_bins, dim3((unsigned)((bins + 3) / 4)), dim3(256), 0, s, m.cnt, list_mb, list_len,
                     nlist, G, B, nwg, gc.nb, m.wpart, m.bbase, m.items);
  RBQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_map_pairs<true>, pg, dim3(256), 0, s, probes, nq, nprobe, gc, nlist, m.cnt, m.bbase,
                     m.fill, m.slots);
  RBQ_HIP(hipGetLastError());
}

int64_t group_map_item_bound(int64_t pairs, int G, int nb, int nlist, int64_t nmb, int64_t max_list_len, int B) {
  if (B <= 0) return pairs / G + (int64_t)nb * nlist + 1;
  const int64_t maxblk = std::max<int64_t>(1, (ceil_div(max_list_len, 64) + B - 1) / B);
  const int64_t sumblk = ceil_div(nmb, B) + nlist;
  return ceil_div(pairs, G) * maxblk + (int64_t)nb * sumblk + 1;
}

int group_map_workgroups(int nlist) { return (nlist + kMapLists - 1) / kMapLists; }

int group_k_steps(int d) { return (d + 63) / 64; }

int group_f8_steps(int d) { return (d + 127) / 128; }

template <bool DUMP>
void launch_scan_group_t(hipStream_t s, const GroupArgs& a, int workgroups, int ks, bool two) {
  if (group_uses_f8(a.bq, a.L.d)) {
    const int ks8 = group_f8_steps(a.L.d);
    RBQ_CHECK(a.qu_ld == 128 * ks8, "fp8 list-major scan: operand rows");
    if (ks8 == 1 && two)
      hipLaunchKernelGGL((k_scan_group<1, QB_F8, 2, DUMP>), dim3(workgroups), dim3(256), 0, s, a);
    else if (ks8 == 1)
      hipLaunchKernelGGL((k_scan_group<1, QB_F8, 4, DUMP>), dim3(workgroups), dim3(256), 0, s, a);
    else if (two)
      hipLaunchKernelGGL((k_scan_group<2, QB_F8, 2, DUMP>), dim3(workgroups), dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((k_scan_group<2, QB_F8, 4, DUMP>), dim3(workgroups), dim3(256), 0, s, a);
    RBQ_HIP(hipGetLastError());
    return;
  }
  RBQ_CHECK(a.qu_ld == a.L.W * 32, "list-major scan: qu rows");
  const int qb = a.bq <= 6 ? QB_DOUBLE : a.bq == 7 ? QB_PLAIN : QB_OFFSET;
#define RBQ_GROUP_LAUNCH_QB(K, QBV)                                                           \
  if (two)                                                                                  \
    hipLaunchKernelGGL((k_scan_group<K, QBV, 2, DUMP>), dim3(workgroups), dim3(256), 0, s, a);    \
  else                                                                                      \
    hipLaunchKernelGGL((k_scan_group<K, QBV, 4, DUMP>), dim3(workgroups), dim3(256), 0, s, a)
#define RBQ_GROUP_LAUNCH(K)                 \
  if (qb == QB_DOUBLE) {                    \
    RBQ_GROUP_LAUNCH_QB(K, QB_DOUBLE);      \
  } else if (qb == QB_PLAIN) {              \
    RBQ_GROUP_LAUNCH_QB(K, QB_PLAIN);       \
  } else {                                  \
    RBQ_GROUP_LAUNCH_QB(K, QB_OFFSET);      \
  }
  switch (ks) {
    case 1: RBQ_GROUP_LAUNCH(1); break;
    case 2: RBQ_GROUP_LAUNCH(2); break;
    case 3: RBQ_GROUP_LAUNCH(3); break;
    default: RBQ_GROUP_LAUNCH(4); break;
  }
#undef RBQ_GROUP_LAUNCH
#undef RBQ_GROUP_LAUNCH_QB
  RBQ_HIP(hipGetLastError());
}

void launch_scan_group(hipStream_t s, const GroupArgs& a, int workgroups) {
  RBQ_CHECK(a.G >= 1 && a.G <= GMAX, "group size out of range");
  const int ks = group_k_steps(a.L.d);
  RBQ_CHECK(ks <= KSMAX, "grouped scan supports d <= 256");
  RBQ_CHECK(a.bq >= 1 && a.bq <= 8, "query bits out of range");
  const bool two = a.G <= 32;
  if (a.dump_ip) {
    launch_scan_group_t<true>(s, a, workgroups, ks, two);
    return;
  }
  launch_scan_group_t<false>(s, a, workgroups, ks, two);
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
