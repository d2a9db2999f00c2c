// Kernel launchers of librbq (host-callable; every kernel is in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rbq {

constexpr int MB = 64;            // vectors per micro-block (one wave64 lane each)
constexpr int MAX_SEL = 4096;     // largest k of a selection (nprobe)
constexpr int MAX_R = 3840;       // largest rerank_n (scan buffer R + 256 <= 4096 keys)

// Device view of the lists of an index.
struct ListsView {
  const uint32_t* blocks;  // micro-block records: W*64 code words, 64 f_add, 64 f_mul
  const int32_t* list_mb;  // [nlist] first micro-block of each list
  const int32_t* list_len; // [nlist] vectors per list
  const int32_t* pos2id;   // [nmb*64] vector id at each position, -1 for padding
  int W;                   // 32-bit code words per vector, ceil(d/32)
  int d;
};

// Per-(query, probe) quantised query: bit-planes [W][BQS] u32, qu bytes [W*32],
// scalars (||r||^2, v_l, Delta, sum qu).
struct PairsView {
  const uint32_t* planes;
  const float4* scal;
  int bqs;                 // plane slots per word (bq rounded up to 4)
};

// C[m][n] = sum_k A[m][k] B[n][k] (mode 0) or bnorm[n] - 2 sum_k A B (mode 1).
// Requires lda, ldb % 4 == 0 and 16-byte aligned rows.
void launch_gemm_tn(hipStream_t s, int mode, const float* A, int lda, const float* B, int ldb,
                    float* C, int ldc, int M, int N, int K, const float* bnorm);

// C[m][n] = sum_k bf16(A[m][k]) bf16(B[n][k]), FP32 accumulation (inputs
// rounded to bfloat16, nearest-even). Same operand rules as launch_gemm_tn.
void launch_gemm_tn_bf16(hipStream_t s, const float* A, int lda, const float* B, int ldb, float* C,
                         int ldc, int M, int N, int K);

// out[m] = min_n key64(bnorm[n] - 2 <A_m, B_n>, n): nearest row of B per row of A.
void launch_assign_argmin(hipStream_t s, const float* A, int lda, const float* B, int ldb,
                          const float* bnorm, int M, int N, int K, uint64_t* out);

// Per row: the k smallest 64-bit keys, ascending (MSB-first radix select, then
// an LDS bitonic sort of the survivors). Keys come from a float matrix (tie =
// column) when `score` is set, else from a key matrix. Pool mode (rowcnt set):
// row r holds its k running keys followed by rowcnt[r] new ones; rows with no
// new keys are skipped, rowcnt[r] is reset to 0 and qthr[r] (if set) is
// lowered to the k-th key's value. An output row may overlap its input row:
// every read of a row precedes every write.
struct TopkArgs {
  const float* score = nullptr;
  const uint64_t* keys = nullptr;
  int64_t ld = 0;              // input row stride
  int ncols = 0;               // keys per row (non-pool mode)
  int k = 0;
  uint64_t* out_keys = nullptr;
  int64_t ldo = 0;             // output row stride (0: k)
  int32_t* out_low = nullptr;  // [rows][k] low word as int32 (-1 for none)
  float* out_val = nullptr;    // [rows][k] high word as float (+inf for none)
  uint32_t* rowcnt = nullptr;
  int max_extra = 0;           // largest rowcnt (pool mode)
  uint32_t* qthr = nullptr;
  const int32_t* rowk = nullptr;  // per-row selection size (<= k); slots past it are untouched
  bool sorted = true;          // false: the k keys in any order (pool merges)
  int merge_threads = 512;     // pool merges: 512 or 256 threads per row (32 keys per thread)
  int KP = 0, cache_cap = 0;   // set by the launcher
};
void launch_row_topk(hipStream_t s, TopkArgs a, int rows);

// Residual r = qrot_i - crot_j for every (query, probe) pair, B_q-bit
// quantisation, bit-planes and scalars; or pack injected qu / scalars.
// qu (optional): [pairs][W*32] bytes in dimension order. qu8 (optional, B_q
// <= 4): [pairs][qu8_ld] fp8 E4M3 bytes of 2 qu in the B-operand order of the
// fp4 x fp8 list-major scan (qu8_ld = 128 ceil(d / 128); see group_qu8_offset).
void launch_quant(hipStream_t s, const float* qrot, int ldq, const float* crot, int ldc,
                  const int32_t* probes, int nq, int nprobe, int d, int W, int bq, int bqs,
                  uint32_t* planes, uint8_t* qu, uint8_t* qu8, int qu8_ld, float4* scal,
                  const uint8_t* inj_qu, const float* inj_scal);

// Code scan with fused estimator and streaming top-R per (query, probe) item.
struct ScanArgs {
  ListsView L;
  PairsView Q;
  const int32_t* probes;   // [nq][nprobe]
  int nq, nprobe, R;
  int p0, pn;              // this launch scans probe ranks [p0, p0 + pn)
  int64_t out_ld;          // keys per query row of `out`: R running keys, then the pool
  uint32_t* pcnt;          // [nq] keys appended to each query's pool
  const uint32_t* qmask;   // if set, only queries with qmask[i] != 0 are scanned
  uint32_t* qthr;          // [nq] ordered-float bound on each query's R-th estimate (or null)
  uint64_t* out;           // candidate rows (est, id) keys
  int32_t* dump_ip;        // debug: [nq][nprobe][maxlen] (or null)
  float* dump_est;
  int64_t maxlen;
  // unquantised-query scan only: rotated queries P^T q and rotated centroids
  // P^T c (row strides ldq, ldc); the residual r = P^T q - P^T c stays FP32
  const float* qrot = nullptr;
  int ldq = 0;
  const float* crot = nullptr;
  int ldc = 0;
};
void launch_scan_popc(hipStream_t s, const ScanArgs& a);

// Query-major scan with the unquantised FP32 residual (Eq.
// rabitq-ip-estimator as the paper's accelerator path evaluates it, no query
// quantisation): per (query, probe) item, E = sum_d b_d r_d by table lookups,
// b_d = +-1, from an LDS table of every sign pattern of each group of 8
// dimensions (4 when d > 128; d <= 1024), then
// d_hat^2 = ||r||^2 + n_x^2 - 2 n_x E / (sqrt(D) alpha_x). Selection, pools
// and dumps (est only) as launch_scan_popc.
void launch_scan_lut(hipStream_t s, const ScanArgs& a);
int scan_lut_max_d();

// Fused query-major scan + per-query selection: one workgroup per query
// scans probe ranks [p0, p0 + pn) and leaves the query's best R (rowk[i] for a
// mixed batch) in out row i's first R slots (unsorted, KEY_NONE padding) with
// the threshold lowered to their R-th estimate. No pool is used.
struct FusedArgs {
  ListsView L;
  PairsView Q;
  const int32_t* probes;   // [nq][nprobe]; -1 = not probed
  int nq, nprobe, R;
  int p0, pn;
  uint64_t* out;           // candidate rows: R running keys first
  int64_t out_ld;
  uint32_t* qthr;
  const int32_t* rowk;     // per-query R (or null)
  const uint32_t* qmask;   // only queries with qmask[i] != 0 (or null: all)
  int reset = 0;           // 1: each query starts afresh (empty running top-R, no threshold)
  int cap = 0;             // set by the launcher
};
void launch_scan_fused(hipStream_t s, FusedArgs a);

// List-major grouped scan on the matrix cores: fp4 x fp8 for B_q <= 4, int8
// otherwise (kernels_group.hip).
struct GroupArgs {
  ListsView L;
  const uint8_t* qu;       // per pair: qu bytes (B_q > 4) or the fp8 operand row (B_q <= 4)
  int qu_ld;               // bytes per pair in qu
  const float4* scal;      // [pairs] (||r||^2, v_l, Delta, sum qu)
  int nq, nprobe, R, nlist, G;
  int bq;                  // query bits B_q
  const int32_t* slots;    // chunk pairs grouped by list
  const int32_t* item_off; // the chunk's item range: [0] first item, [1] end
  const int4* items;       // per item: (list's first micro-block, first slot, pairs, list length)
  uint32_t* item_counter;  // work-queue cursor, zero before the launch
  const uint32_t* qthr;    // per-query threshold (ordered float of d_hat^2)
  uint64_t* pool;          // candidate rows: R running keys then the pool
  int64_t pool_ld;
  int cap;                 // pool capacity per query
  uint32_t* pcnt;          // [nq] pool fill
  uint32_t* overflow;      // [nq] set when a query's pool overflowed
  uint32_t* any_overflow;  // set with any overflow flag
  const int32_t* probes = nullptr;  // [nq][nprobe] (the debug dumps place positions by list)
  int32_t* dump_ip = nullptr;  // debug: [pairs][maxlen] ip and d_hat^2 of every estimate (or null)
  float* dump_est = nullptr;
  int64_t maxlen = 0;
};
int group_k_steps(int d);
// The fp4 x fp8 form of the list-major scan (B_q <= 4): 128-dimension steps
// per pair, and the bytes per pair of its operand rows.
int group_f8_steps(int d);
inline bool group_uses_f8(int bq, int d) { return bq <= 4 && d <= 256; }
// Byte offset, in a pair's 128-byte fp8 operand row of one step, of the two
// bytes for dimensions 8 l + j and 8 l + j + 4 of the step (l = 0..15, j =
// 0..3). The scan's fp4 A operand gives lane group g the bits of code word g
// of the step with dimension 32 g + 4 i + q at element k = 32 g + 8 q + i
// (nibble i of dword q); the matrix core reads B elements k in [16 g, 16 g +
// 16) from bytes [32 g, 32 g + 16) of lane group g and k in [64 + 16 g, 80 +
// 16 g) from bytes [32 g + 16, 32 g + 32), so the byte for dimension 32 g +
// 4 i + q sits where that k is read; the two dimensions 4 apart are
// neighbouring k and share a 16-bit word. For every l the offsets of j = 1,
// 2, 3 exceed that of j = 0 by 8, 32 and 40.
__host__ __device__ inline int group_qu8_offset(int l, int j) {
  const int k = 32 * (l >> 2) + 8 * j + 2 * (l & 3);
  return k < 64 ? 32 * (k >> 4) + (k & 15) : 32 * ((k - 64) >> 4) + 16 + ((k - 64) & 15);
}
// The list-major chunks of a search: probe ranks [bound[0], bound[nb]), chunk
// c = [bound[c], bound[c+1]).
constexpr int kMaxGroupChunks = 16;
struct GroupChunks {
  int nb = 0;
  int bound[kMaxGroupChunks + 1] = {};
};
// Pairs of every list-major chunk grouped by (chunk, list) and cut into items:
// item = (first micro-block of its index block, first slot, pairs, vectors of
// the block), an index block being B micro-blocks of the list (B = 0: the
// whole list) and an item up to G pairs. Buffers: cnt, fill and bbase hold
// nb * nlist words (cnt and fill zero on entry); wpart 2 * nb *
// group_map_workgroups(nlist) words; chunk_items nb + 1 words (the item range
// of chunk c is [chunk_items[c], chunk_items[c + 1])); slots one word per
// pair; items at most group_map_item_bound(...) entries.
struct GroupMap {
  int32_t* cnt;
  int32_t* fill;
  int32_t* bbase;
  int32_t* wpart;
  int32_t* chunk_items;
  int32_t* slots;
  int4* items;
};
int group_map_workgroups(int nlist);
int64_t group_map_item_bound(int64_t pairs, int G, int nb, int nlist, int64_t nmb, int64_t max_list_len, int B);
void launch_group_map(hipStream_t s, const int32_t* probes, int nq, int nprobe, const GroupChunks& gc,
                      int nlist, int G, int B, const int32_t* list_mb, const int32_t* list_len,
                      const GroupMap& m);
void launch_scan_group(hipStream_t s, const GroupArgs& a, int workgroups);
void launch_reset_masked(hipStream_t s, const uint32_t* mask, uint64_t* rows, int64_t ld, int R,
                         uint32_t* qthr, uint32_t* pcnt, int nq);

// IVF-Flat list-major scan (kernels_flat.hip): exact squared distances
// ||q||^2 + ||x||^2 - 2 <q, x> of full-precision vectors on the FP32 matrix
// cores, items and pools as the list-major code scan's.
struct FlatArgs {
  const float* blocks;     // per micro-block: dp rows of 64 floats, then 64 squared norms
  const int32_t* pos2id;
  int d;
  const float* q;          // queries, row stride ldq
  int ldq;
  int nq, nprobe, R, G;
  const int32_t* slots;
  const int32_t* item_off;
  const int4* items;
  uint32_t* item_counter;
  const uint32_t* qthr;
  uint64_t* pool;
  int64_t pool_ld;
  int cap;
  uint32_t* pcnt;
  uint32_t* overflow;
  uint32_t* any_overflow;
};
int flat_dp(int d);  // rows per flat record: round_up(d, 4)
// Fills the flat records of micro-blocks [0, nmb) from id-ordered rows of X.
void launch_flat_fill(hipStream_t s, const float* X, int ldx, const int32_t* pos2id, int64_t nmb, int d,
                      float* out);
void launch_scan_flat(hipStream_t s, const FlatArgs& a, int workgroups);

// Exact re-rank: per query, gather the candidates' raw vectors, exact squared
// L2 in FP32, top-k by (distance, id). Output rows have stride k; with rowk
// set, row i keeps its best rowk[i] (<= k) and pads the rest with (-1, +inf).
void launch_rerank(hipStream_t s, const float* q, int ldq, const float* X, int64_t n, int ldx,
                   int d, const uint64_t* cand, int64_t ldc, int nq, int R, int k, int64_t* ids,
                   float* dist, const int32_t* rowk = nullptr);

// The same with byte rows (raw vectors that are integers 0..255, held exactly):
// the per-lane order of the sums is the FP32 kernel's, so results are equal.
void launch_rerank_u8(hipStream_t s, const float* q, int ldq, const uint8_t* X, int64_t n, int ldx,
                      int d, const uint64_t* cand, int64_t ldc, int nq, int R, int k, int64_t* ids,
                      float* dist, const int32_t* rowk = nullptr);
// Counts the elements of X (rows x d, stride ld) that are not integers in
// [0, 255]; converts `total` floats to bytes.
void launch_count_not_u8(hipStream_t s, const float* X, int64_t rows, int d, int ld, unsigned* out);
void launch_to_u8(hipStream_t s, const float* X, int64_t total, uint8_t* out);

// probes[i][p] = -1 for p >= qnp[i] (a query that probes fewer lists than the
// batch's widest one); scans and maps skip such pairs.
void launch_mask_probes(hipStream_t s, int32_t* probes, int nq, int nprobe, const int32_t* qnp);

// RaBitQ encoder (FP64): one launch encodes micro-blocks [mb_begin, mb_end).
void launch_encode(hipStream_t s, const float* X, int ldx, const float* C, int ldc,
                   const float* Pt, int ldp, const int32_t* pos2id, const int32_t* mb_list,
                   int64_t mb_begin, int64_t mb_end, int d, int W, uint32_t* blocks,
                   float* nx_out, float* alpha_out);

// out[r][i] = sum_d A[r][d] P[d][i] in FP64, rounded to FP32 (Pt = P^T rows);
// also nrm[r] = ||A_r||^2 (FP64 -> FP32) if nrm is set.
void launch_rotate_rows_f64(hipStream_t s, const float* A, int lda, const float* Pt, int ldp,
                            int rows, int d, float* out, int ldo, float* nrm);

// Per-search state: cand rows [nq][R] (stride cand_ld) = KEY_NONE, qthr =
// ~0, pcnt = 0, overflow = 0 (if set), z0[0..n0) = 0, f2[0..n2) = ~0.
struct SearchInit {
  uint64_t* cand = nullptr;
  int64_t cand_ld = 0;
  int nq = 0, R = 0;
  uint32_t* qthr = nullptr;
  uint32_t* pcnt = nullptr;
  uint32_t* overflow = nullptr;
  uint32_t* z0 = nullptr;
  int64_t n0 = 0;
  uint32_t* f2 = nullptr;  // f2[0..n2) = 0xFFFFFFFF
  int64_t n2 = 0;
};
void launch_search_init(hipStream_t s, const SearchInit& a);

void launch_fill_u32(hipStream_t s, uint32_t* p, uint32_t v, int64_t n);
void launch_fill_u64(hipStream_t s, uint64_t* p, uint64_t v, int64_t n);
void launch_fill_rows_u64(hipStream_t s, uint64_t* p, int64_t ld, int64_t rows, int cols, uint64_t v);
void launch_gather_rows(hipStream_t s, const float* X, int ldx, const int64_t* idx, int64_t n,
                        float* out, int ldo);

// k-means++ on the device: one step adds centre j (row `pick` of T) and updates
// the running min distances and per-block sums; the choose step samples the
// next centre with probability proportional to the min distance.
void launch_kpp_update(hipStream_t s, const float* T, int ldt, int64_t n, int d,
                       const int64_t* pick, float* mind, double* blocksum, int first);
void launch_kpp_choose(hipStream_t s, const float* mind, const double* blocksum, int64_t n,
                       double u, int64_t* pick);
void launch_copy_row(hipStream_t s, const float* T, int ldt, const int64_t* pick, float* dst,
                     int d);

}  // namespace rbq
