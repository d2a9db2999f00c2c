#!/usr/bin/env python3
"""Benchmark of batched IVF-RaBitQ search on one MI355X.

Workload (default ``sift10m``): 10M x 128 integer-valued skewed vectors,
nlist 4096, batches of 1024 queries, B_q 4, k 10. A step is one pass of the
whole search path over one batch: probe GEMM + top-nprobe, query rotation,
residual quantisation, code scan with the fused estimator, per-query top-R,
exact re-rank. The operating point (nprobe, rerank_n) is the fastest measured
point whose recall@10 against exact kNN reaches 0.95: the workload's listed
points first, then a wider grid; ``--nprobe``/``--rerank`` fix it instead.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "QPS at recall@10>=0.95 (1 GPU), code-scan HBM GB/s vs peak, p50/p99 ms"
HBM_PEAK_GBS = 8000.0
# 32-bit VALU lane-ops of MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (no packed FP32)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU operations the estimator epilogue needs per (query, vector) once the
# integer inner product is known: 2 ip - sum(qu), int->float, two products and
# a sum for E, (||r||^2 + n_x^2), the factor product and its sum, the threshold
# compare
EPILOGUE_OPS = 9
# PMC summaries (HBM bytes per launch of a scan kernel at one operating point)
_CSRC = os.path.join(ROOT, "paper_2605_16007_amd", "csrc")
# kernel -> (its PMC summary, the sources whose concatenation's sha256 the
# summary records: the kernel's file and the two headers it includes)
PMC_SUMMARIES = {
    "k_scan_group": (os.path.join(ROOT, "profiles", "k_scan_group_sift10m_pmc.md"),
                     [os.path.join(_CSRC, f) for f in ("kernels_group.hip", "kernels.hpp", "common.hpp")]),
    "k_scan_popc": (os.path.join(ROOT, "profiles", "k_scan_popc_unit96_50m.md"),
                    [os.path.join(_CSRC, f) for f in ("kernels.hip", "kernels.hpp", "common.hpp")]),
}


def source_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel, point):
    """HBM bytes per launch of `kernel` from its committed PMC summary, if the
    kernel source has not changed since the counters were taken and they were
    taken at this operating point (e.g. "sift10m nprobe=512 rerank=3840")."""
    import re
    summary, srcs = PMC_SUMMARIES[kernel]
    try:
        text = open(summary).read()
        sha = source_sha(srcs)
    except OSError:
        return None
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
    t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    o = re.search(r"operating_point:\s*(.+)", text)
    if not m or not t or not o or m.group(1) != sha or o.group(1).strip() != point:
        return None
    return float(t.group(1))


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------------- CPU baseline

_CPU_STATE = {}


def _oracle_chunk(task):
    """Worker: the oracle's search of one chunk of queries (one BLAS thread)."""
    from threadpoolctl import threadpool_limits
    import oracle as O
    i, nprobe, k, R = task
    st = _CPU_STATE
    with threadpool_limits(1):
        t = time.perf_counter()
        O.search(st["idx"], st["X"], st["Q"][st["chunks"][i]], nprobe, k, R)
        return time.perf_counter() - t


class CpuBaseline:
    """The oracle as it stands, on the host cores, over a bounded sample.

    Sample: the first ``nqueries`` queries of the batch, searched by the oracle
    on an oracle-built index over the first 2.5M database rows with nlist
    scaled so that lists hold as many vectors as in the full workload
    (N / nlist); each query therefore probes and scans the same number of
    vectors as on the full index (up to nprobe = that nlist). Index construction is not timed. The worker processes are
    forked here, before the GPU is used, and run the sample later at the
    operating point the GPU run settles on.
    """

    def __init__(self, w, Q, nqueries, cores):
        import multiprocessing as mp
        import oracle as O
        from synth import database
        self.w, self.nqueries, self.cores = w, nqueries, cores
        self.n_sub = min(w.n, 2_500_000)
        self.nlist_sub = max(1, int(round(w.nlist * self.n_sub / w.n)))
        t = time.perf_counter()
        Xs = database(w, 0, self.n_sub)
        rng = np.random.default_rng(0)
        C = O.kmeans(Xs, self.nlist_sub, rng, iters=3, restarts=1, train_n=64 * self.nlist_sub)
        idx = O.build(Xs, self.nlist_sub, bq=w.bq, centroids=C, rng=rng)
        log(f"[cpu_baseline] oracle index over {self.n_sub} rows, nlist {self.nlist_sub}: "
            f"{time.perf_counter() - t:.1f}s")
        self.chunks = np.array_split(np.arange(nqueries), cores)
        _CPU_STATE.update(idx=idx, X=Xs, Q=Q[:nqueries], chunks=self.chunks)
        self.pool = mp.get_context("fork").Pool(cores)

    def run(self, nprobe, k, R):
        # the sub-index has nlist_sub lists: beyond that, time nprobe = nlist_sub
        # and scale by the number of vectors scanned per query (extrapolated)
        npc = min(nprobe, self.nlist_sub)
        scale = npc / nprobe
        t = time.perf_counter()
        per = self.pool.map(_oracle_chunk, [(i, npc, k, R) for i in range(len(self.chunks))])
        wall = time.perf_counter() - t
        one_core = len(self.chunks[0]) / per[0] * scale if per[0] > 0 else None
        w = self.w
        value = self.nqueries / wall * scale
        log(f"[cpu_baseline] nprobe {npc} rerank {R}: {self.nqueries / wall:.1f} q/s on "
            f"{self.cores} cores; reported {value:.2f} q/s at nprobe {nprobe}")
        extra = "" if scale == 1 else (
            f"; timed at nprobe {npc} (every list of the sub-index) and scaled by {scale:.4f} "
            f"to nprobe {nprobe} in proportion to vectors scanned (extrapolated)")
        return {
            "value": value, "unit": "queries/s", "cores": self.cores, "kind": "oracle",
            "sample": (f"first {self.nqueries} queries of the batch; oracle index over the first "
                       f"{self.n_sub} rows with nlist {self.nlist_sub} (same {w.n // w.nlist} "
                       f"vectors per list on average as the full workload; centroids from 3 "
                       f"Lloyd iterations), nprobe {nprobe}, k {k}, rerank {R}; FP64 NumPy, one "
                       f"BLAS thread per worker process; index construction not timed{extra}"),
            "extrapolated": scale != 1, "one_core_qps": one_core, "wall_s": wall,
        }

    def close(self):
        self.pool.close()
        self.pool.join()


# ----------------------------------------------------------------- ground truth

def exact_knn_gpu(Xt, Qt, X_host, Q_host, k, shortlist=64, chunk=0):
    """Exact kNN for recall: FP32 GEMM shortlist on the GPU with plain torch
    ops, then FP64 re-ranking of the shortlist on the host."""
    import torch
    nq = Qt.shape[0]
    chunk = chunk or max(1 << 14, min(1 << 20, (1 << 28) // max(1, nq)))  # <= 1 GiB of distances
    qn = (Qt * Qt).sum(1, keepdim=True)
    best_v = torch.full((nq, 0), float("inf"), device=Qt.device)
    best_i = torch.zeros((nq, 0), dtype=torch.int64, device=Qt.device)
    for s in range(0, Xt.shape[0], chunk):
        xb = Xt[s:s + chunk]
        d = qn - 2.0 * (Qt @ xb.T) + (xb * xb).sum(1)[None, :]
        v, i = torch.topk(d, min(shortlist, xb.shape[0]), dim=1, largest=False)
        best_v = torch.cat([best_v, v], 1)
        best_i = torch.cat([best_i, i + s], 1)
        v, o = torch.topk(best_v, min(shortlist, best_v.shape[1]), dim=1, largest=False)
        best_v, best_i = v, torch.gather(best_i, 1, o)
    cand = best_i.cpu().numpy()
    gt = np.empty((nq, k), np.int64)
    for q in range(nq):
        c = cand[q]
        dd = np.sum((X_host[c].astype(np.float64) - Q_host[q].astype(np.float64)) ** 2, axis=1)
        o = np.lexsort((c, dd))[:k]
        gt[q] = c[o]
    return gt


def recall(ids, gt):
    k = gt.shape[1]
    return float(np.mean([len(set(a[:k]) & set(b)) / k for a, b in zip(ids.tolist(), gt.tolist())]))


# ----------------------------------------------------------------- main

def serve_compare(idx, w, args):
    """Open-loop Poisson traces on the resident index: the continuous-batching
    server against plain one-query-at-a-time search (rbq_search, nq = 1, in
    arrival order), both driven by the library's native replay. Per request
    nprobe ~ U{8, 16, ..., 256}, k ~ U{10, 100}, rerank_n = 10 k. The two return
    identical results (checked here), so their recall is equal."""
    from paper_2605_16007_amd import Server
    from synth import arrivals, queries
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    counts = [max(64, min(args.serve_max, int(r * args.serve_seconds))) for r in rates]
    Qs = queries(w, max(counts))
    out = {"workload": f"{w.name} index, Poisson arrivals, nprobe U{{8..256 step 8}}, "
                       f"k U{{10,100}}, rerank_n 10k",
           "server": {"lanes": 2, "max_batch": 1024, "mem_budget_gib": 1.0}, "rates": {}}

    def summary(n, arr, lat):
        done = arr + lat
        return {"qps": n / float(done.max() - arr[0]), "p50_ms": float(np.percentile(lat, 50)) * 1e3,
                "p99_ms": float(np.percentile(lat, 99)) * 1e3}

    with Server(idx, lanes=2, max_batch=1024, max_nprobe=256, max_k=100, max_rerank=1000,
                mem_budget=1 << 30) as srv:
        t, npb, kk = arrivals(rates[0], 256, seed=99)
        srv.replay(Qs[:256], npb, kk, 10 * kk, np.zeros(256))  # warm-up
        idx.replay_plain(Qs[:32], npb[:32], kk[:32], 10 * kk[:32], np.zeros(32))
        for ri, (rate, n) in enumerate(zip(rates, counts)):
            t, npb, kk = arrivals(rate, n, seed=ri)
            t = t - t[0]
            before = srv.stats()
            ids_s, d_s, lat_s = srv.replay(Qs[:n], npb, kk, 10 * kk, t)
            after = srv.stats()
            ids_p, d_p, lat_p = idx.replay_plain(Qs[:n], npb, kk, 10 * kk, t)
            batches = after["batches"] - before["batches"]
            rec = {"requests": n, "trace_s": float(t[-1]),
                   "server": dict(summary(n, t, lat_s), mean_batch=n / max(1, batches)),
                   "plain": summary(n, t, lat_p),
                   "identical_results": bool(np.array_equal(ids_s, ids_p) and np.array_equal(d_s, d_p))}
            out["rates"][str(int(rate))] = rec
            log(f"[serving] {rate:.0f} q/s x {n}: server {rec['server']['qps']:.0f} q/s "
                f"p50 {rec['server']['p50_ms']:.2f} p99 {rec['server']['p99_ms']:.2f} ms "
                f"(batch {rec['server']['mean_batch']:.1f}); plain {rec['plain']['qps']:.0f} q/s "
                f"p50 {rec['plain']['p50_ms']:.2f} p99 {rec['plain']['p99_ms']:.2f} ms; "
                f"identical {rec['identical_results']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--streams", type=int, default=1,
                    help="HIP streams the timed batches alternate over (each batch whole on one)")
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="sift10m")
    ap.add_argument("--nprobe", type=int, default=0,
                    help="fix nprobe (default: the fastest point reaching recall@10 >= 0.95)")
    ap.add_argument("--rerank", type=int, default=0, help="fix rerank_n (with --nprobe)")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="finish with one device-to-device copy of this size (PMC calibration)")
    ap.add_argument("--n", type=int, default=0, help="database rows (default: the workload's)")
    ap.add_argument("--batches", type=int, default=4, help="distinct query batches cycled")
    ap.add_argument("--latency-iters", type=int, default=50)
    ap.add_argument("--cpu-queries", type=int, default=128)
    ap.add_argument("--cpu-cores", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rotation", choices=("fp32", "bf16"), default="fp32",
                    help="query rotation precision (bf16: BF16 inputs, FP32 accumulation)")
    ap.add_argument("--vectors-on-host", action="store_true",
                    help="keep the raw vectors in pinned host memory and re-rank on host cores")
    ap.add_argument("--no-autotune", action="store_true", help="time the built-in launch rule")
    ap.add_argument("--tune-cache", default="",
                    help="autotune cache file: loaded if it exists (no tuning runs), else written")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the timing of both scan forms at the chosen point")
    ap.add_argument("--scan", choices=("auto", "popcount", "mfma"), default="auto",
                    help="force the scan form of the timed loop (auto: tuned per chunk)")
    ap.add_argument("--serve-rates", default="5000,10000,20000,50000",
                    help="Poisson arrival rates (queries/s) of the serving comparison; '' skips it")
    ap.add_argument("--serve-seconds", type=float, default=0.5,
                    help="seconds of arrivals per rate (capped by --serve-max)")
    ap.add_argument("--serve-max", type=int, default=8000, help="most requests per rate")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures the search path on one GPU only; this build runs no "
              "multi-GPU configuration (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    from synth import get, database, queries
    w = get(args.workload)
    if args.n:
        w = w.with_(n=args.n, nlist=max(1, int(round(w.nlist * args.n / w.n))))
    nb = args.batches
    t = time.perf_counter()
    X = database(w)
    Qall = queries(w, w.nq * nb)
    log(f"[data] {w.name}: {w.n} x {w.d} + {nb} x {w.nq} queries in {time.perf_counter() - t:.1f}s")

    cpu_pool = None
    if not args.no_cpu_baseline:
        # forked before the GPU is touched
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        cpu_pool = CpuBaseline(w, Qall[:w.nq], args.cpu_queries, cores)

    import torch
    from paper_2605_16007_amd import Index
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t = time.perf_counter()
    idx = Index.build(X, w.nlist, bq=w.bq, seed=w.seed, vectors_on_host=args.vectors_on_host)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    info = idx.info()
    idx.set_option("rotation", 1 if args.rotation == "bf16" else 0)
    log(f"[build] {build_s:.1f}s, max list {info['max_list_len']}, codes {info['code_bytes'] / 1e6:.1f} MB")

    Qb = [torch.from_numpy(Qall[i * w.nq:(i + 1) * w.nq]).to(dev) for i in range(nb)]
    Xt = torch.from_numpy(X).to(dev)
    gt = exact_knn_gpu(Xt, Qb[0], X, Qall[:w.nq], w.k)
    del Xt
    torch.cuda.empty_cache()

    # Operating point: the listed (nprobe, rerank_n) first; if none reaches
    # recall@10 >= 0.95, wider probes and longer re-rank lists are tried, and
    # the fastest point that reaches it is timed.
    assign = idx.export("assign")
    gt_lists = assign[gt]

    def probe_recall(npb):
        pr = idx.search_debug(Qall[:w.nq], npb, w.k, w.rerank_n, want={"probes"})["probes"]
        return float(np.mean([np.isin(gl, p).mean() for gl, p in zip(gt_lists, pr)]))

    def eval_point(npb, R):
        ids, _ = idx.search(Qb[0], npb, w.k, R)
        torch.cuda.synchronize()
        return recall(ids.cpu().numpy(), gt)

    def quick_qps(npb, R, steps=8):
        ids_ = torch.empty((w.nq, w.k), dtype=torch.int64, device=dev)
        dd_ = torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)
        idx.search(Qb[0], npb, w.k, R, ids=ids_, dists=dd_)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in range(steps):
            idx.search(Qb[s % nb], npb, w.k, R, ids=ids_, dists=dd_)
        torch.cuda.synchronize()
        return w.nq * steps / (time.perf_counter() - t)

    rec, prec = {}, {}
    points = [(p, args.rerank or w.rerank_n) for p in ((args.nprobe,) if args.nprobe else w.nprobe)]
    for pt in points:
        rec[pt] = eval_point(*pt)
        prec[pt[0]] = probe_recall(pt[0])
        log(f"[recall] nprobe {pt[0]} rerank {pt[1]}: recall@{w.k} = {rec[pt]:.4f} "
            f"(probe recall {prec[pt[0]]:.4f})")
    ok = [pt for pt in points if rec[pt] >= 0.95]
    if not ok and not args.nprobe:
        # longer re-rank lists at every probe count whose probed lists hold
        # >= 95% of the true neighbours (listed counts first, then wider ones)
        top = min(w.nlist, 4096)
        wider = [p for p in (256, 512, 1024, 2048) if max(w.nprobe) < p <= top]
        for npb in list(w.nprobe) + wider:
            if npb not in prec:
                prec[npb] = probe_recall(npb)
            if prec[npb] < 0.95:
                continue
            for R in sorted({min(3840, f * w.rerank_n) for f in (2, 5, 10, 20, 40)}):
                pt = (npb, R)
                rec[pt] = eval_point(*pt)
                log(f"[recall] nprobe {npb} rerank {R}: recall@{w.k} = {rec[pt]:.4f} "
                    f"(probe recall {prec[npb]:.4f})")
                if rec[pt] >= 0.95:
                    ok.append(pt)
                    break
    if args.nprobe:
        nprobe, R = points[0]
    elif ok:
        qq = {pt: quick_qps(*pt) for pt in ok}
        nprobe, R = max(ok, key=lambda pt: qq[pt])
        log("[choose] " + ", ".join(f"{pt}: {q:.0f} q/s" for pt, q in qq.items()))
    else:
        nprobe, R = max(rec, key=lambda pt: rec[pt])
        log(f"[choose] no point reached recall 0.95; timing the best one {(nprobe, R)}")
    # the autotuner picks the launch choices of each timed shape (results are
    # unchanged by construction and checked by the library)
    tuned = {}
    loaded = 0
    if args.tune_cache and os.path.exists(args.tune_cache):
        loaded = idx.tune_load(args.tune_cache)
        log(f"[autotune] {loaded} tuned shapes loaded from {args.tune_cache}")
        tuned = {"loaded_from_cache": loaded}
    if not args.no_autotune and not loaded:
        for pt in ([(p, w.rerank_n) for p in w.nprobe] if not args.nprobe else []) + [(nprobe, R)]:
            tuned[f"nprobe={pt[0]},rerank={pt[1]}"] = idx.autotune(Qb[0], pt[0], w.k, pt[1])
            log(f"[autotune] {pt}: {tuned[f'nprobe={pt[0]},rerank={pt[1]}']}")
        if args.tune_cache:
            idx.tune_save(args.tune_cache)
    listed_qps = {f"{p}": quick_qps(p, w.rerank_n) for p in w.nprobe} if not args.nprobe else {}

    idx.set_option("scan", {"auto": 0, "popcount": 1, "mfma": 2}[args.scan])
    ids = torch.empty((w.nq, w.k), dtype=torch.int64, device=dev)
    dd = torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)
    # consecutive batches alternate over a few streams (a search never waits
    # for the host, so one batch's kernels can fill the CUs another's leave
    # idle); each stream has its own outputs
    nst = max(1, args.streams)
    streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
    outs = [(torch.empty((w.nq, w.k), dtype=torch.int64, device=dev),
             torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)) for _ in range(nst)]

    def step(s):
        st = streams[s % nst]
        oi, od = outs[s % nst]
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=oi, dists=od, stream=st.cuda_stream)

    torch.cuda.synchronize()
    for s in range(args.warmup):
        step(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(s)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / args.steps
    qps = w.nq * args.steps / elapsed
    # stage times, scanned work and per-launch kernel times: the same searches
    # again with the library's instrumentation on (events and counting kernels
    # of their own, kept out of the timed steps above)
    idx.set_timing(True)
    for s in range(min(args.steps, 10)):
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=ids, dists=dd)
    torch.cuda.synchronize()
    tm = idx.timings()
    idx.set_timing(False)

    # latency per batch (one synchronised batch at a time)
    lat = []
    for s in range(args.latency_iters):
        torch.cuda.synchronize()
        t = time.perf_counter()
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=ids, dists=dd)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # the two scan forms at the chosen point
    variants = {}
    if not args.no_variants:
        for name, mode in (("popcount_query_major", 1), ("mfma_list_major", 2)):
            idx.set_option("scan", mode)
            variants[name] = quick_qps(nprobe, R, steps=10)
        idx.set_option("scan", 0)
        log("[variants] " + ", ".join(f"{k_}: {v:.0f} q/s" for k_, v in variants.items()))

    serving = serve_compare(idx, w, args) if args.serve_rates else None

    cpu = cpu_pool.run(nprobe, w.k, R) if cpu_pool else None
    if cpu_pool:
        cpu_pool.close()

    ns = max(1, tm["searches"])
    wname = w.name if not args.n else f"{w.name}/n={w.n}"  # the workload as the PMC summaries name it
    scan_s = tm["scan_ms"] / ns * 1e-3
    if tm["group_launches"] > 0:
        # list-major matrix-core scan (the dominant kernel): bound by the VALU epilogue
        launches = tm["group_launches"] / ns
        gscan_s = tm["group_scan_ms"] / ns * 1e-3
        gvec = tm["group_vectors"] / ns
        achieved = gvec * EPILOGUE_OPS / gscan_s / 1e12
        traffic = pmc_traffic("k_scan_group", f"{wname} nprobe={nprobe} rerank={R}")
        roofline = {"kernel": "k_scan_group", "bound": "alu", "achieved": achieved,
                    "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                    "traffic": traffic,
                    "launches_per_step": launches,
                    "avg_launch_ms": gscan_s * 1e3 / launches,
                    "estimates_per_launch": gvec / launches,
                    "read_bytes_per_launch": tm["group_read_bytes"] / ns / launches,
                    "read_gbs": tm["group_read_bytes"] / ns / gscan_s / 1e9,
                    "schedule_gbs_effective": gvec * (4 * ((w.d + 31) // 32) + 8) / gscan_s / 1e9,
                    "other_scan_ms_per_step": (scan_s - gscan_s) * 1e3}
    else:
        launches = max(1, tm["popc_launches"]) / ns
        achieved = tm["read_bytes"] / ns / scan_s / 1e9
        roofline = {"kernel": "k_scan_popc", "bound": "hbm", "achieved": achieved,
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                    "traffic": pmc_traffic("k_scan_popc",
                                           f"{wname} nprobe={nprobe} rerank={R} scan={args.scan}"),
                    "launches_per_step": launches,
                    "avg_launch_ms": scan_s * 1e3 / launches,
                    "bytes_per_launch": tm["read_bytes"] / ns / launches}
    if args.calibrate_copy_gib > 0:
        nb = int(args.calibrate_copy_gib * (1 << 30)) // 4
        a = torch.ones(nb, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[calibrate] copied {nb * 4} bytes device to device")
        del a, b

    line = {
        "metric": METRIC,
        "value": qps,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the list-major scan's matrix-core operands (fp4 codes x fp8 2 qu for
        # B_q <= 4, int8 above; d > 256 has none), the query-major popcounts,
        # and the fp32 estimator
        "dtype": ("fp4 x fp8 MFMA" if w.bq <= 4 and w.d <= 256 else "i8 MFMA" if w.d <= 256 else "no MFMA")
                 + " / u32 popcount + fp32",
        "scan_form": args.scan,
        "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "nlist": w.nlist, "nprobe": nprobe,
                   "batch": w.nq, "k": w.k, "rerank_n": R, "bq": w.bq,
                   "rotation": args.rotation,
                   "rerank_on": "host" if args.vectors_on_host else "gpu",
                   "streams": nst, "parallelism": "none (1 GPU)"},
        "recall_at_10": rec[(nprobe, R)],
        "recall_by_point": {f"nprobe={p},rerank={r}": v for (p, r), v in rec.items()},
        "probe_recall_by_nprobe": {str(p): v for p, v in prec.items()},
        "qps_at_listed_nprobe": listed_qps,
        "qps_by_scan_form": variants,
        "autotune": tuned,
        "p50_ms": p50,
        "p99_ms": p99,
        "stage_ms": {s: tm[f"{s}_ms"] / ns for s in
                     ("probe", "rotate", "quant", "scan", "merge", "rerank", "total")},
        "roofline": roofline,
        "serving": serving,
        "cpu_baseline": cpu,
        "build_s": build_s,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
