/*
 * rbq.h — C ABI of librbq, an IVF-RaBitQ vector search library for AMD
 * MI355X (gfx950).
 *
 * The library builds an IVF index whose lists hold 1-bit RaBitQ codes plus two
 * FP32 factors per vector (Sec. 2.2.1), and answers batches of k-nearest-
 * neighbour queries under squared L2 distance (Sec. 2.1.1) in the paper's
 * search phases (Sec. 3.1.2): probe the nprobe nearest lists, estimate the
 * distance of every vector in them from its code (Eqs. rabitq-ip-estimator,
 * approx-dist), keep the rerank_n best estimates, re-rank those by exact
 * distance and return the k best.
 *
 * Conventions for every entry point:
 *   - Every call returns an rbq_status; nothing throws across the ABI.
 *     On failure rbq_last_error() returns a message (thread-local, valid until
 *     the next call on the same thread).
 *   - Argument errors return RBQ_EINVAL before any side effect.
 *   - Pointers marked "host or device" may point to host memory or to device
 *     memory of the index's GPU; the library tells them apart with
 *     hipPointerGetAttributes. The caller owns every buffer it passes.
 *   - Matrices are row-major, float32, rows of d values, no padding.
 *   - Distances are squared L2. Results rank by (distance, id) ascending; when
 *     fewer than k candidates exist the rest is padded with id -1 and
 *     distance +inf.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream). Calls on
 *     one index may run concurrently on distinct streams. When a call returns,
 *     host outputs are complete; device outputs are complete in stream order.
 */
#ifndef RBQ_H
#define RBQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBQ_OK = 0,
  RBQ_EINVAL = -1,   /* bad argument; nothing was changed */
  RBQ_ENOMEM = -2,   /* device or host allocation failed */
  RBQ_EDEVICE = -3,  /* a HIP runtime call failed */
  RBQ_ESTATE = -4,   /* object in the wrong state (e.g. server stopped) */
  RBQ_EAGAIN = -5    /* try again later (serving queue full) */
} rbq_status;

typedef struct rbq_index rbq_index; /* opaque; owns its device and host copies */

/* Index construction parameters (Sec. 3.1.1). Fill with rbq_build_params_init. */
typedef struct {
  int32_t nlist;           /* number of IVF lists, 1..n */
  int32_t bq;              /* query quantisation bits B_q, 1..8 (default 4) */
  uint64_t seed;           /* seeds the library's own random draws */
  int32_t kmeans_iters;    /* Lloyd iterations limit (default 25) */
  int32_t kmeans_restarts; /* k-means runs, lowest objective kept (default 3) */
  int64_t train_n;         /* k-means training rows; 0 = min(n, 256*nlist) */
  const float* rotation;   /* optional host d*d orthogonal P, row-major; NULL:
                              the library draws a Haar-random P from `seed` */
  const float* centroids;  /* optional host nlist*d centroids; NULL: k-means */
  const int32_t* assignment; /* optional host n list ids in [0,nlist); NULL:
                              nearest centroid */
  int32_t vectors_on_host; /* where the raw vectors of the exact re-rank live
                              (Sec. 3.3.4): 0 HBM (GPU re-rank); 1 host memory
                              (re-rank on host cores; the index's own copy is
                              2 MiB-aligned and advised for transparent huge
                              pages, not pinned: only host threads read it);
                              -1 (default) automatic: HBM when, with the index
                              built, they leave at least max(8 GiB, 1/8 of the
                              device) of device memory free, else host memory */
  int32_t host_threads;    /* host re-rank threads (0: min(16, hardware
                              threads), less two from 8 up, leaving cores to
                              the threads that queue GPU work) */
  int32_t borrow_vectors;  /* 1: when the vectors end on the host, the index
                              keeps the caller's rows instead of a copy: x must
                              then be host memory (pageable or pinned) holding
                              n*d float32, and the caller keeps it unchanged
                              until rbq_free_index. Rows backed by 2 MiB pages
                              (madvise MADV_HUGEPAGE) re-rank fastest. EINVAL
                              with vectors_on_host = 0 or a device x */
  int32_t ivf_flat;        /* 1: also keep every list's full-precision vectors
                              in HBM, in list order (d <= 256), for the IVF-Flat
                              scan (RBQ_OPT_ESTIMATOR 2, the comparison system
                              of Sec. 4.2); not saved by rbq_save */
  int32_t kmeans_init;     /* 0: k-means++ seeding (default); 1: nlist distinct
                              training rows drawn uniformly, the random initial
                              centroids of Sec. 3.1.1 Phase 1 (no sequential
                              seeding pass: for very large nlist) */
  int32_t reserved[3];     /* must be zero */
} rbq_build_params;

void rbq_build_params_init(rbq_build_params* p);

/*
 * Build an index over x (host or device, n*d float32), Sec. 3.1.1: IVF
 * centroids (given or k-means on a training sample, Phases 1-2), assignment of
 * every vector to its nearest centroid (Sec. 2.1.2), random orthogonal P, and
 * the RaBitQ encoding of each vector against its centroid (Phase 3;
 * Eqs. normalized-residual, quantize, rabitq-alpha). The index copies x
 * (unless it borrows x, see borrow_vectors); the build itself stages all n
 * rows in device memory. Errors: EINVAL for n < 1, d < 1, nlist outside
 * [1,n], bq outside [1,8], non-finite inputs, a bad assignment, a bad
 * vectors_on_host / borrow_vectors combination; ENOMEM; EDEVICE.
 */
rbq_status rbq_build_index(const float* x, int64_t n, int32_t d, const rbq_build_params* p,
                           rbq_index** out);

rbq_status rbq_free_index(rbq_index* idx);

typedef struct {
  int64_t n;
  int32_t d, nlist, bq, vectors_on_host;  /* vectors_on_host as placed: 0 or 1 */
  int64_t max_list_len;      /* largest list */
  int64_t device_bytes;      /* device memory held by the index */
  int64_t code_bytes;        /* packed codes + factors on the device */
  int32_t vectors_borrowed;  /* 1: the host rows are the caller's (borrow_vectors) */
  int32_t reserved;
} rbq_index_info;

rbq_status rbq_get_info(const rbq_index* idx, rbq_index_info* info);

/*
 * Search a batch (Sec. 3.1.2 Phases 1-5). q: host or device nq*d float32.
 * ids: host or device nq*k int64; sqdist: host or device nq*k float32.
 * Requires 1 <= nprobe <= min(nlist, 4096), 1 <= k <= rerank_n <= 3840,
 * nq >= 0 (nq = 0 is a no-op). Errors: EINVAL for argument errors, ENOMEM,
 * EDEVICE. The library allocates per-call device scratch, reused across calls.
 */
rbq_status rbq_search(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                      int32_t rerank_n, int64_t* ids, float* sqdist, void* stream);

/*
 * For callers that cannot allocate device memory (work recorded under stream
 * capture, serving loops that forbid allocation): rbq_search whose device
 * workspace is a fixed 256 MiB array inside the library, one per GPU, held
 * from the first call on that GPU until the process ends. The call allocates
 * no device or pinned host memory and creates no events. q, ids and sqdist
 * must be device pointers; the index must keep its raw vectors in HBM
 * (vectors_on_host 0). Results equal rbq_search's. The candidate pool is
 * sized to fit the array, so a large batch may take more chunks than with
 * rbq_search. Errors: as rbq_search, and EINVAL for host pointers, a host
 * re-rank index, or a batch whose smallest workspace exceeds the array (the
 * message gives its size; split the batch). Calls that overlap on one GPU
 * (concurrent streams or threads) share the array and race: the caller
 * serialises them.
 */
rbq_status rbq_search_noalloc(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                              int32_t rerank_n, int64_t* ids, float* sqdist, void* stream);

/*
 * Mixed batch: the batch-processing search of Sec. 3.1.2 in which query i uses
 * its own nprobe[i], k[i] and rerank_n[i] (host int32 arrays of nq, each in the
 * ranges rbq_search accepts). Query i's result is the same as rbq_search of
 * that query alone with its parameters: probing, estimates, the top-rerank_n
 * selection and the re-rank are per query, and no kernel's arithmetic depends
 * on the rest of the batch. ids / sqdist (host or device) hold nq rows of
 * k_stride (>= every k[i]) values; row i has its k[i] results, then
 * (-1, +inf).
 */
rbq_status rbq_search_mixed(rbq_index* idx, const float* q, int64_t nq, const int32_t* nprobe,
                            const int32_t* k, const int32_t* rerank_n, int32_t k_stride,
                            int64_t* ids, float* sqdist, void* stream);

/* Canonical exports (host dst, exactly `bytes` long), all in vector-id order. */
enum {
  RBQ_EXPORT_CENTROIDS = 1,  /* nlist*d float32 */
  RBQ_EXPORT_ROTATION = 2,   /* d*d float32, row-major P (z = P^T r) */
  RBQ_EXPORT_ASSIGN = 3,     /* n int32 list ids */
  RBQ_EXPORT_CODES = 4,      /* n*ceil(d/8) uint8, LSB-first: dim j in byte j>>3 bit j&7 */
  RBQ_EXPORT_FACTORS = 5,    /* n*2 float32: (n_x = ||x-c||, alpha_x) */
  RBQ_EXPORT_LIST_SIZES = 6  /* nlist int64 */
};
rbq_status rbq_export(const rbq_index* idx, int32_t what, void* dst, size_t bytes);

/*
 * Stage-by-stage search for parity checks: the same kernels as rbq_search,
 * with optional injected inputs and per-stage outputs. All pointers here are
 * HOST pointers; NULL skips the item. Layouts (pair = query*nprobe + rank):
 *   inject_probes  nq*nprobe int32     probed lists used instead of probing
 *   inject_qu      nq*nprobe*d uint8   quantised residual qu (needs scalars)
 *   inject_scalars nq*nprobe*3 float32 (||r||^2, v_l, Delta) per pair
 *   probes         nq*nprobe int32;  probe_score nq*nprobe float32
 *                  (||c||^2 - 2<q,c>, the ranking score; ||q||^2 omitted)
 *   qrot           nq*d float32 (P^T q)
 *   qu             nq*nprobe*d uint8; scalars nq*nprobe*4 float32
 *                  (||r||^2, v_l, Delta, sum qu)
 *   ip, est        nq*nprobe*max_list_len int32 / float32: per probed list,
 *                  the integer inner product and estimated d_hat^2 of its
 *                  vectors in ascending-id order (unused slots zero)
 *   cand_ids, cand_est nq*rerank_n int64 / float32: the coarse top-rerank_n
 *   ids, sqdist    nq*k final results
 *   probe_chunk    scan at most this many probe ranks per launch, merging
 *                  the running top-rerank_n after each (0: as rbq_search)
 */
typedef struct {
  const int32_t* inject_probes;
  const uint8_t* inject_qu;
  const float* inject_scalars;
  int32_t* probes;
  float* probe_score;
  float* qrot;
  uint8_t* qu;
  float* scalars;
  int32_t* ip;
  float* est;
  int64_t* cand_ids;
  float* cand_est;
  int64_t* ids;
  float* sqdist;
  int32_t probe_chunk;  /* probe ranks per scan launch (0 = automatic) */
  int32_t reserved;
  const float* inject_qrot; /* nq*d float32 rotated queries P^T q used instead of
                               the rotation's (the residuals of both estimators
                               are formed from them) */
} rbq_debug_io;

rbq_status rbq_search_debug(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                            int32_t rerank_n, rbq_debug_io* io);

/* Stage timing with HIP events recorded on each call's stream. While timing
 * is enabled every rbq_search adds its stage times to running sums; reading
 * them waits for the recorded events. rbq_set_timing(idx, 1) clears the sums
 * and enables timing; rbq_set_timing(idx, 0) disables it. Stages:
 * probe (score GEMM + top-nprobe), rotate (P^T q GEMM), quant (residual
 * quantisation), scan (the code-scan kernel alone), merge (per-query top-R),
 * rerank (exact re-rank); total spans probe..rerank. */
typedef struct {
  int64_t searches;          /* timed searches summed */
  float probe_ms, rotate_ms, quant_ms, scan_ms, merge_ms, rerank_ms, total_ms;
  int64_t scanned_vectors;   /* sum over (query, probed list) of list sizes: the
                                estimated distances computed */
  int64_t scan_bytes;        /* scanned_vectors * (4*ceil(d/32) + 8): code and factor
                                bytes if every (query, list) pair read its list */
  int64_t read_bytes;        /* code and factor bytes the scan kernels' schedule reads
                                (list-major items read a list once per item) */
  int64_t group_launches;    /* list-major scan launches summed */
  int64_t popc_launches;     /* query-major scan launches (popcount or fused) summed */
  float group_scan_ms;       /* the list-major scan launches alone */
  int64_t group_vectors;     /* scanned_vectors of the list-major launches */
  int64_t group_read_bytes;  /* read_bytes of the list-major launches */
  int64_t fused_launches;    /* of popc_launches: the fused scan-and-select launches */
  float fused_scan_ms;       /* the fused launches alone */
  int32_t reserved;
  int64_t fused_vectors;     /* scanned_vectors of the fused launches */
  int64_t fused_read_bytes;  /* read_bytes of the fused launches */
  int64_t redo_queries;      /* queries whose list-major pool overflowed and
                                were searched again from scratch (exact) */
} rbq_timings;

rbq_status rbq_set_timing(rbq_index* idx, int32_t enabled);
rbq_status rbq_get_timings(rbq_index* idx, rbq_timings* t);

/*
 * Serving loop: continuous batching over a resident index (the batch
 * processing of Sec. 3.1.2 with requests that arrive one at a time).
 *
 * Requests are submitted one query at a time, from any host thread, each with
 * its own nprobe, k and rerank_n. A server runs `lanes` host threads, each with
 * its own HIP stream and a device workspace of mem_budget bytes allocated at
 * creation. A lane that is free takes the oldest waiting requests, in arrival
 * order, for as long as the batch stays within max_batch queries and its
 * workspace need (probe scores, quantised residuals and candidate rows, which
 * grow with the batch's size, nprobe and rerank_n) within mem_budget; runs them
 * as one mixed batch (rbq_search_mixed); and publishes each request's result.
 * Requests that arrive while batches are on the device join the next batch a
 * lane forms, and with lanes > 1 that batch is launched while earlier ones
 * still run, so their kernels overlap on the device. Each result equals that
 * of rbq_search of the query alone with its own parameters.
 *
 * A server must be destroyed before its index. rbq_submit / rbq_poll /
 * rbq_wait may be called concurrently from several threads.
 */
typedef struct rbq_server rbq_server; /* opaque */

typedef struct {
  int32_t lanes;        /* batches in flight at once, 1..8 (default 2) */
  int32_t max_batch;    /* queries per batch, 1..65536 (default 1024) */
  int32_t queue_cap;    /* requests held at once, waiting, running or finished
                           but not yet collected, 1..2^22 (default 65536) */
  int32_t max_nprobe;   /* largest nprobe of a request (0 = default: min(nlist, 256)) */
  int32_t max_k;        /* largest k (default 100) */
  int32_t max_rerank;   /* largest rerank_n (default 1000) */
  int64_t mem_budget;   /* device workspace bytes per lane (default 1 GiB) */
  int32_t reserved[8];  /* must be zero */
} rbq_server_params;

typedef struct {
  int64_t submitted;      /* requests accepted by rbq_submit */
  int64_t rejected;       /* rbq_submit calls refused with RBQ_EAGAIN */
  int64_t completed;      /* results published (including failed batches) */
  int64_t batches;        /* batches run */
  int64_t max_batch_seen; /* largest batch run */
  int64_t budget_cuts;    /* batches closed because the next request would have
                             taken the workspace need past mem_budget */
  int64_t reserved[2];
} rbq_server_stats;

rbq_status rbq_server_params_init(rbq_server_params* p);
/* Allocates the lanes' streams, workspaces and pinned staging buffers and
 * starts the lane threads. ENOMEM if an allocation fails. */
rbq_status rbq_server_create(rbq_index* idx, const rbq_server_params* p, rbq_server** out);
/* Queues one query (host pointer, d floats, copied before return). EINVAL for
 * parameters outside the server's limits, ENOMEM if the request alone needs
 * more than mem_budget, EAGAIN when queue_cap requests are held, ESTATE after
 * destroy began. */
rbq_status rbq_submit(rbq_server* srv, const float* q, int32_t nprobe, int32_t k, int32_t rerank_n,
                      uint64_t* ticket);
/* Non-blocking. *done = 0: not finished, outputs untouched. *done = 1: ids and
 * sqdist (host, the request's k values) hold the result and the ticket is
 * released. If the request's batch failed, its status is returned instead
 * (with the message) and the ticket is released. latency_ns (optional)
 * receives submit-to-result time. EINVAL for an unknown or released ticket. */
rbq_status rbq_poll(rbq_server* srv, uint64_t ticket, int64_t* ids, float* sqdist, int32_t* done,
                    int64_t* latency_ns);
/* As rbq_poll, waiting up to timeout_us (< 0: no limit); EAGAIN on time-out. */
rbq_status rbq_wait(rbq_server* srv, uint64_t ticket, int64_t* ids, float* sqdist,
                    int64_t timeout_us, int64_t* latency_ns);
rbq_status rbq_server_get_stats(rbq_server* srv, rbq_server_stats* st);
/* Finishes every queued and running request, stops the lanes and frees the
 * server (uncollected results are dropped). */
rbq_status rbq_server_destroy(rbq_server* srv);

/* An open-loop arrival trace and where its results go (all host memory). */
typedef struct {
  const float* q;          /* n*d queries */
  const int32_t* nprobe;   /* n values each */
  const int32_t* k;
  const int32_t* rerank_n;
  const double* arrival_s; /* n non-decreasing arrival times, seconds after the start */
  int64_t* ids;            /* n*k_stride results, padded with (-1, +inf) past k[i] */
  float* sqdist;
  double* latency_s;       /* n: time the result was ready minus arrival time */
  int64_t n;
  int32_t k_stride;        /* >= every k[i] */
  int32_t reserved;        /* must be zero */
} rbq_replay_io;

/* Replays the trace through the server: request i is submitted at its arrival
 * time (if the queue is full, as soon as a request has been collected; its
 * latency still counts from the arrival time) and collected by a second host
 * thread. Returns when every result is in. */
rbq_status rbq_server_replay(rbq_server* srv, const rbq_replay_io* io);
/* The same trace served one query at a time, in arrival order, by rbq_search
 * with nq = 1 on one stream of the calling thread (the plain per-query form
 * the serving loop is compared with). */
rbq_status rbq_replay_plain(rbq_index* idx, const rbq_replay_io* io);

/* Tuning options of an index (apply to later searches on any thread). None
 * changes a search's results except RBQ_OPT_ROTATION.
 *   RBQ_OPT_SCAN        0: choose per chunk of probe ranks (default; or as
 *                          autotuned): with d <= 256, the list-major scan for
 *                          chunks whose (query, probed list) pairs number
 *                          >= RBQ_OPT_GROUP_MIN * nlist, the query-major scan
 *                          for the others,
 *                       1: query-major popcount scan only,
 *                       2: list-major matrix-core scan for every chunk (d <= 256),
 *                       3: one work item per query: a workgroup per query scans
 *                          and selects over all its probes in one launch
 *                          (batches of >= 128 queries with d <= 1024; else 1)
 *   RBQ_OPT_GROUP_MIN   the threshold above (default 4: each list is probed
 *                       by >= 4 queries of the chunk on average)
 *   RBQ_OPT_POOL_CAP    cap on the per-query pool of the list-major scan
 *                       (0 = the workspace bound; small values exercise the
 *                       overflow path, which stays exact)
 *   RBQ_OPT_ROTATION    query rotation P^T q: 0 FP32 (default), 1 BF16 inputs
 *                       with FP32 accumulation (q and P rounded to bfloat16,
 *                       nearest-even; changes the estimates slightly)
 *   RBQ_OPT_GROUP_SIZE  queries per list-major work item, 1..64 (0 = as
 *                       autotuned, else 64); items of up to 32 queries take
 *                       two 16-query matrix-core tiles, larger ones four
 *   RBQ_OPT_ESTIMATOR   0 (default): the residual is quantised to B_q bits
 *                       (Sec. 2.2.2); 1: unquantised, E = sum_d b_d r_d with
 *                       r the FP32 rotated residual, as the paper's
 *                       accelerator path computes it (Eq.
 *                       rabitq-ip-estimator, Sec. 4.3); query-major scan with
 *                       sign-pattern tables of 8-dimension groups (4 when
 *                       d > 128), d <= 1024; changes the estimates. In this
 *                       mode rbq_search_debug does not fill qu and scalars,
 *                       and ip holds nothing; 2: IVF-Flat (an index built
 *                       with ivf_flat): exact squared distances of the
 *                       full-precision vectors of the probed lists on the FP32
 *                       matrix cores (||q||^2 + ||x||^2 - 2<q,x>), the best
 *                       rerank_n re-ranked exactly as usual (rerank_n = k
 *                       gives plain IVF-Flat); list-major scan only. A query
 *                       whose candidate pool would overflow fails the search
 *                       (RBQ_ENOMEM) instead of returning a wrong result
 *   RBQ_OPT_BLOCK       list-major work items cover index blocks of this many
 *                       64-vector micro-blocks of a list (Sec. 3.3.1), so a
 *                       long list is shared out over several workgroups;
 *                       0: whole lists; -1 (default): as autotuned, else 0
 *   RBQ_OPT_HOST_PARTS  sub-batches of a search whose re-rank runs on host
 *                       cores (Sec. 3.3.4: the host re-ranks one while the GPU
 *                       searches the next), 1..64; 0 (default): 4 for batches
 *                       of >= 2048 queries, 2 for >= 256, else 1, halved while
 *                       a sub-batch would probe each list fewer than 8 times
 *                       on average. rbq_autotune tunes for the sub-batch size
 *                       in force when it runs */
enum { RBQ_OPT_SCAN = 1, RBQ_OPT_GROUP_MIN = 2, RBQ_OPT_POOL_CAP = 3, RBQ_OPT_ROTATION = 4,
       RBQ_OPT_GROUP_SIZE = 5, RBQ_OPT_ESTIMATOR = 6, RBQ_OPT_BLOCK = 7, RBQ_OPT_HOST_PARTS = 8 };
rbq_status rbq_set_option(rbq_index* idx, int32_t option, int64_t value);

/*
 * Autotuner (the launch schedule of Sec. 3.3.1 adapted per batch shape).
 * Some launch choices of a search leave its results unchanged: the scan form
 * of each chunk of probe ranks (query-major popcount or the list-major
 * matrix-core scan), the queries grouped per list-major work item (G), the persistent
 * workgroups per compute unit, and the sizes of the chunks. rbq_autotune times every
 * candidate on the given queries (host or device, nq x d; representative of
 * later batches) over three searches (one when the first already takes 1.5x
 * the best time so far), checks that each returns the same results, and stores the
 * fastest for the bucket of (nq, nprobe, rerank_n) rounded up to powers of
 * two. Later searches of any shape in a tuned bucket use it (an explicit
 * RBQ_OPT_SCAN still fixes the scan form). Blocks the calling thread.
 * The table can be saved to / loaded from a text cache; its entries are keyed
 * by device architecture, d, B_q, nlist, n and the list-size histogram, and
 * only matching entries load. For an index whose raw vectors are on the host,
 * where a search runs on the GPU in sub-batches (RBQ_OPT_HOST_PARTS) while
 * host cores re-rank the previous one, the choices are tuned (on the GPU
 * phases alone) and stored for the sub-batch size in force.
 */
typedef struct {
  int32_t scan;          /* 1 query-major popcount only; 2 list-major matrix core for the
                            chunks of probe ranks selected by chunk_group_min */
  int32_t group_size;    /* queries per list-major item */
  int32_t wg_per_cu;     /* persistent list-major workgroups per compute unit */
  int32_t first_factor;  /* first chunk: ~first_factor * rerank_n candidates per query */
  float ms;              /* time per search with the chosen launch choices */
  float ms_default;      /* time per search with the built-in rule */
  int32_t trials;        /* candidate configurations timed */
  int32_t chunk_group_min; /* a chunk is list-major when its (query, probe) pairs
                              number >= this * nlist (0: every chunk) */
  int32_t growth;        /* each chunk after the first is (growth - 1) x the probe
                            ranks already scanned */
  int32_t early_form;    /* chunks before the list-major ones, in batches of >= 128
                            queries: 0 one workgroup per query scans and selects;
                            1 popcount scan per (query, probe), then a merge */
  int32_t block;         /* list-major items cover index blocks of this many
                            micro-blocks (0: whole lists), tuned after the above */
  int32_t merge_form;    /* pool merges on 256-thread workgroups instead of 512:
                            0 none, 1 all but the first list-major chunk's, 2 all;
                            tuned last */
} rbq_tune_result;

rbq_status rbq_autotune(rbq_index* idx, const float* q, int64_t nq, int32_t nprobe, int32_t k,
                        int32_t rerank_n, rbq_tune_result* out);
rbq_status rbq_tune_save(rbq_index* idx, const char* path);
rbq_status rbq_tune_load(rbq_index* idx, const char* path, int32_t* loaded);
rbq_status rbq_tune_clear(rbq_index* idx);

/* Persist / restore an index (versioned binary with per-section checksums). */
rbq_status rbq_save(const rbq_index* idx, const char* path);
rbq_status rbq_load(const char* path, rbq_index** out);

const char* rbq_last_error(void);
const char* rbq_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RBQ_H */
