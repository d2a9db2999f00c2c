#!/usr/bin/env python3
"""Benchmark of batched IVF-RaBitQ search on one MI355X.

Headline workload (default): the whole 400M x 96 unit-vector mixture (nlist
65,536; ``--shard`` takes its first 50M rows with nlist 8192 instead, the same
list length), batches of 10,000 queries, B_q 4, k 10; the raw vectors live in
host memory (2 MiB pages) that the index borrows and the exact re-rank runs on
host cores, overlapped with the GPU search of the other batches in flight
(the split into host sub-batches and the number of batches in flight, two
or three, are picked by a short trial). The whole
set is built with k-means from nlist random training rows, 10 Lloyd
iterations and one run (the objective changes by under 1e-4 after the
seventh), and its recall is measured on 1,000 queries. A step is one pass of the whole search path over one batch:
probe GEMM + top-nprobe, query rotation, residual quantisation, code scan with
the fused estimator, per-query top-R, exact re-rank. The operating point
(nprobe, rerank_n) is the fastest measured point whose recall@10 against exact
kNN reaches 0.95: the workload's listed points first, then longer re-rank
lists and wider probes; ``--nprobe``/``--rerank`` fix it instead.

Secondary workload (default ``sift10m``: 10M x 128 integer-valued vectors,
nlist 4096, batches of 1024, raw vectors in HBM, GPU re-rank): the same
measurement, an ablation of GPU against host re-rank, and the serving
comparison (continuous batching against one query at a time).

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
# rows of the 400M x 96 workload's shard (one eighth: nlist 8192)
SHARD_ROWS = 50_000_000
# PMC summaries: profiles/<kernel>_<workload>.md record the HBM bytes per
# launch of one scan kernel at one operating point, with the sha256 of the
# kernel's source file and the two headers it includes
_CSRC = os.path.join(ROOT, "paper_2605_16007_amd", "csrc")
KERNEL_SOURCES = {
    "k_scan_group": [os.path.join(_CSRC, f) for f in ("kernels_group.hip", "kernels.hpp", "common.hpp")],
    "k_scan_popc": [os.path.join(_CSRC, f) for f in ("kernels.hip", "kernels.hpp", "common.hpp")],
    "k_scan_fused": [os.path.join(_CSRC, f) for f in ("kernels.hip", "kernels.hpp", "common.hpp")],
}


def source_sha(paths):
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel, point):
    """HBM bytes per launch of `kernel` from a committed PMC summary taken at
    this operating point (e.g. "sift10m nprobe=512 rerank=3840") for the
    current kernel source; None if there is none."""
    import glob
    import re
    try:
        sha = source_sha(KERNEL_SOURCES[kernel])
    except (KeyError, OSError):
        return None
    for summary in sorted(glob.glob(os.path.join(ROOT, "profiles", f"{kernel}_*.md"))):
        text = open(summary).read()
        m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", text)
        t = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
        o = re.search(r"operating_point:\s*(.+)", text)
        if m and t and o and m.group(1) == sha and o.group(1).strip() == point:
            return float(t.group(1))
    return None


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
    nprobe ~ U{8, 16, ..., 256}, k ~ U{10, 100}, rerank_n = 10 k. Each rate's
    trace starts with ``serve_warmup_s`` seconds of arrivals that are served but
    not counted. The plain form replays the first ``plain_max`` requests of the
    same trace (it saturates far below the offered rates). Both forms return
    identical results on the requests they share (checked here), so their
    recall is equal."""
    from paper_2605_16007_amd import Server
    from synth import arrivals, queries
    rates = [float(r) for r in args.serve_rates.split(",") if r]
    counts = [max(64, min(args.serve_max, int(r * args.serve_seconds))) for r in rates]
    warms = [int(r * args.serve_warmup_s) for r in rates]
    Qs = queries(w, max(c + m for c, m in zip(counts, warms)))
    out = {"workload": f"{w.name} index, Poisson arrivals, nprobe U{{8..256 step 8}}, "
                       f"k U{{10,100}}, rerank_n 10k",
           "server": {"lanes": 2, "max_batch": 1024, "mem_budget_gib": 1.0}, "rates": {}}

    def summary(arr, lat):
        done = arr + lat
        return {"requests": len(arr), "qps": len(arr) / float(done.max() - arr[0]),
                "p50_ms": float(np.percentile(lat, 50)) * 1e3,
                "p99_ms": float(np.percentile(lat, 99)) * 1e3}

    with Server(idx, lanes=2, max_batch=1024, max_nprobe=256, max_k=100, max_rerank=1000,
                mem_budget=1 << 30) as srv:
        t, npb, kk = arrivals(rates[0], 256, seed=99)
        srv.replay(Qs[:256], npb, kk, 10 * kk, np.zeros(256))  # first-use warm-up
        idx.replay_plain(Qs[:32], npb[:32], kk[:32], 10 * kk[:32], np.zeros(32))
        for ri, (rate, n, wm) in enumerate(zip(rates, counts, warms)):
            tot = n + wm
            t, npb, kk = arrivals(rate, tot, seed=ri)
            t = t - t[0]
            before = srv.stats()
            ids_s, d_s, lat_s = srv.replay(Qs[:tot], npb, kk, 10 * kk, t)
            after = srv.stats()
            m = min(tot, args.plain_max)
            ids_p, d_p, lat_p = idx.replay_plain(Qs[:m], npb[:m], kk[:m], 10 * kk[:m], t[:m])
            batches = after["batches"] - before["batches"]
            pw = min(wm, m // 2)
            rec = {"offered_qps": rate, "warmup_requests": wm, "trace_s": float(t[-1] - t[wm]),
                   "server": dict(summary(t[wm:], lat_s[wm:]), mean_batch=tot / max(1, batches)),
                   "plain": summary(t[pw:m], lat_p[pw:]),
                   "identical_results": bool(np.array_equal(ids_s[:m], ids_p) and np.array_equal(d_s[:m], d_p))}
            out["rates"][str(int(rate))] = rec
            log(f"[serving] {rate:.0f} q/s, {n} requests after {wm} warm-up: server "
                f"{rec['server']['qps']:.0f} q/s p50 {rec['server']['p50_ms']:.2f} p99 "
                f"{rec['server']['p99_ms']:.2f} ms (batch {rec['server']['mean_batch']:.1f}); plain "
                f"({m} requests) {rec['plain']['qps']:.0f} q/s p50 {rec['plain']['p50_ms']:.2f} "
                f"p99 {rec['plain']['p99_ms']:.2f} ms; identical {rec['identical_results']}")
    return out


# ----------------------------------------------------------------- one workload

def roofline_of(tm, w, wname, nprobe, R, scan):
    """Per-launch figures of the scan kernels from one instrumented pass.

    Achieved bandwidth counts the bytes each kernel's item schedule reads at
    least once (the code and factor records: a list-major item reads its list
    once for its group of queries, a query-major item once for its query)
    divided by that kernel's HIP-event time. The dominant kernel (the most scan
    time per batch) is the one reported; the others sit under "forms"."""
    ns = max(1, tm["searches"])
    rec = 4 * ((w.d + 31) // 32) + 8
    forms = {}
    g_ms = tm["group_scan_ms"] / ns
    f_ms = tm["fused_scan_ms"] / ns
    p_ms = tm["scan_ms"] / ns - g_ms - f_ms
    g_l = tm["group_launches"] / ns
    f_l = tm["fused_launches"] / ns
    p_l = (tm["popc_launches"] - tm["fused_launches"]) / ns
    parts = {
        "k_scan_group": (g_l, g_ms, tm["group_read_bytes"] / ns, tm["group_vectors"] / ns),
        "k_scan_fused": (f_l, f_ms, tm["fused_read_bytes"] / ns, tm["fused_vectors"] / ns),
        "k_scan_popc": (p_l, p_ms, (tm["read_bytes"] - tm["group_read_bytes"] - tm["fused_read_bytes"]) / ns,
                        (tm["scanned_vectors"] - tm["group_vectors"] - tm["fused_vectors"]) / ns),
    }
    for name, (launches, ms, byts, vecs) in parts.items():
        if launches <= 0 or ms <= 0:
            continue
        gbs = byts / (ms * 1e-3) / 1e9
        f = {"launches_per_step": launches, "avg_launch_ms": ms / launches,
             "schedule_bytes_per_launch": byts / launches, "achieved_gbs": gbs,
             "frac_hbm": gbs / HBM_PEAK_GBS, "estimates_per_launch": vecs / launches,
             "ms_per_step": ms}
        if name == "k_scan_group":
            alu = vecs * EPILOGUE_OPS / (ms * 1e-3) / 1e12
            f["alu"] = {"ops_per_estimate": EPILOGUE_OPS, "achieved_tops": alu, "peak_tops": VALU_PEAK_TOPS,
                        "frac": alu / VALU_PEAK_TOPS}
            # every (query, vector) pair as if each read its own record
            f["pair_bytes_gbs_effective"] = vecs * rec / (ms * 1e-3) / 1e9
        forms[name] = f
    if not forms:
        return None
    dom = max(forms, key=lambda n: forms[n]["ms_per_step"])
    d = forms[dom]
    point = f"{wname} nprobe={nprobe} rerank={R}" + ("" if dom == "k_scan_group" else f" scan={scan}")
    return {"kernel": dom, "bound": "hbm", "achieved": d["achieved_gbs"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["frac_hbm"], "traffic": pmc_traffic(dom, point),
            "launches_per_step": d["launches_per_step"], "avg_launch_ms": d["avg_launch_ms"],
            "bytes_per_launch": d["schedule_bytes_per_launch"], "forms": forms}


def alternating_qps(idx, Qb, nprobe, k, R, n_streams, steps):
    """Queries/s of `steps` searches issued from this thread, batch s on
    stream s mod n_streams (each stream with its own outputs)."""
    import torch
    dev = Qb[0].device
    sts = [torch.cuda.Stream(device=dev) for _ in range(n_streams)]
    outs = [(torch.empty((Qb[0].shape[0], k), dtype=torch.int64, device=dev),
             torch.empty((Qb[0].shape[0], k), dtype=torch.float32, device=dev)) for _ in range(n_streams)]

    def go(count):
        for s in range(count):
            idx.search(Qb[s % len(Qb)], nprobe, k, R, ids=outs[s % n_streams][0],
                       dists=outs[s % n_streams][1], stream=sts[s % n_streams].cuda_stream)
    go(n_streams)
    torch.cuda.synchronize()
    t = time.perf_counter()
    go(steps)
    torch.cuda.synchronize()
    return Qb[0].shape[0] * steps / (time.perf_counter() - t)


def measure(w, args, *, host_vectors, role, points_hint=None, cpu_pool=None):
    """Build the index of workload ``w``, choose its operating point, time it.
    Returns the fields of one result line (``role`` names it in the log)."""
    import torch
    from paper_2605_16007_amd import Index, huge_page_rows
    from synth import database, get, queries
    dev = torch.device("cuda:0")
    nb = args.batches
    t = time.perf_counter()
    if host_vectors:
        # raw vectors drawn straight into huge-page host memory that the index
        # borrows (no second host copy)
        X = huge_page_rows(w.n, w.d)
        database(w, out=X)
    else:
        X = database(w)
    Qall = queries(w, w.nq * nb)
    gen_s = time.perf_counter() - t
    log(f"[{role}] {w.name}: {w.n} x {w.d} + {nb} x {w.nq} queries in {gen_s:.1f}s")
    t = time.perf_counter()
    kw = {}
    if args.kmeans_iters:
        kw["kmeans_iters"] = args.kmeans_iters
    if args.kmeans_restarts:
        kw["kmeans_restarts"] = args.kmeans_restarts
    if args.train_n:
        kw["train_n"] = args.train_n
    if args.kmeans_init:
        kw["kmeans_init"] = args.kmeans_init
    idx = Index.build(X, w.nlist, bq=w.bq, seed=w.seed,
                      vectors_on_host=host_vectors, borrow_vectors=host_vectors,
                      ivf_flat=not args.no_flat and w.d <= 256, **kw)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    info = idx.info()
    idx.set_option("rotation", 1 if args.rotation == "bf16" else 0)
    log(f"[{role}] build {build_s:.1f}s, max list {info['max_list_len']}, codes "
        f"{info['code_bytes'] / 1e6:.1f} MB, vectors on host {info['vectors_on_host']} "
        f"(borrowed {info['vectors_borrowed']})")

    Qb = [torch.from_numpy(Qall[i * w.nq:(i + 1) * w.nq]).to(dev) for i in range(nb)]
    gt_n = min(w.nq, args.gt_queries)
    t = time.perf_counter()
    Xt = torch.from_numpy(X).to(dev)
    gt = exact_knn_gpu(Xt, Qb[0][:gt_n], X, Qall[:gt_n], w.k)
    del Xt
    torch.cuda.empty_cache()
    log(f"[{role}] exact kNN of {gt_n} queries in {time.perf_counter() - t:.1f}s")
    assign = idx.export("assign")
    gt_lists = assign[gt]

    def probe_recall(npb):
        pr = idx.search_debug(Qall[:gt_n], npb, w.k, w.rerank_n, want={"probes"})["probes"]
        return float(np.mean([np.isin(gl, p).mean() for gl, p in zip(gt_lists, pr)]))

    def eval_point(npb, R):
        ids, _ = idx.search(Qb[0], npb, w.k, R)
        torch.cuda.synchronize()
        return recall(ids[:gt_n].cpu().numpy(), gt)

    # batches in flight at once: with the re-rank on host cores a search
    # returns only when its host re-rank is done, so a second caller thread
    # (own stream, own workspace) keeps the GPU busy meanwhile
    conc = args.concurrency if args.concurrency > 0 else (2 if host_vectors else 1)

    def quick_qps(npb, R, steps=8, threads=1):
        """Queries/s of `steps` searches issued from `threads` caller threads,
        each on its own stream."""
        import threading
        sts = [torch.cuda.Stream(device=dev) for _ in range(threads)]
        bufs = [(torch.empty((w.nq, w.k), dtype=torch.int64, device=dev),
                 torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)) for _ in range(threads)]

        def run(t, first, count):
            torch.cuda.set_device(dev)
            for s in range(first + t, first + count, threads):
                idx.search(Qb[s % nb], npb, w.k, R, ids=bufs[t][0], dists=bufs[t][1],
                           stream=sts[t].cuda_stream)

        def all_threads(first, count):
            th = [threading.Thread(target=run, args=(t, first, count)) for t in range(threads)]
            for x in th:
                x.start()
            for x in th:
                x.join()
        all_threads(0, threads)
        torch.cuda.synchronize()
        t = time.perf_counter()
        all_threads(0, steps)
        torch.cuda.synchronize()
        return w.nq * steps / (time.perf_counter() - t)

    # Operating point: the listed (nprobe, rerank_n) first; if none reaches
    # recall@10 >= 0.95, longer re-rank lists at every probe count whose probed
    # lists hold >= 95% of the true neighbours, and the fastest point reaching
    # it is timed.
    rec, prec = {}, {}
    fixed = args.nprobe and role == "headline"
    points = [(args.nprobe, args.rerank or w.rerank_n)] if fixed else [(p, w.rerank_n) for p in w.nprobe]
    for pt in points + (points_hint or []):
        rec[pt] = eval_point(*pt)
        prec.setdefault(pt[0], probe_recall(pt[0]))
        log(f"[{role}] nprobe {pt[0]} rerank {pt[1]}: recall@{w.k} = {rec[pt]:.4f} "
            f"(probe recall {prec[pt[0]]:.4f})")
    ok = [pt for pt in rec if rec[pt] >= 0.95]
    if not ok and not fixed:
        top = min(w.nlist, 4096)
        wider = [p for p in (256, 512, 1024, 2048) if max(w.nprobe) < p <= top]
        for npb in list(w.nprobe) + wider:
            if npb not in prec:
                prec[npb] = probe_recall(npb)
            if prec[npb] < 0.95:
                continue
            lo = w.rerank_n if rec.get((npb, w.rerank_n), 1.0) < 0.95 else 0
            for R in sorted({min(3840, f * w.rerank_n) for f in (2, 3, 4, 5, 7, 10, 15, 20, 40)}):
                pt = (npb, R)
                rec[pt] = eval_point(*pt)
                log(f"[{role}] nprobe {npb} rerank {R}: recall@{w.k} = {rec[pt]:.4f} "
                    f"(probe recall {prec[npb]:.4f})")
                if rec[pt] >= 0.95:
                    # the smallest rerank_n (to 5% or 10) between the last
                    # grid point that missed and this one
                    hi = R
                    while lo and hi - lo > max(10, hi // 20):
                        mid = (lo + hi) // 20 * 10
                        if not lo < mid < hi:
                            break
                        rec[(npb, mid)] = eval_point(npb, mid)
                        log(f"[{role}] nprobe {npb} rerank {mid}: recall@{w.k} = {rec[(npb, mid)]:.4f}")
                        if rec[(npb, mid)] >= 0.95:
                            hi = mid
                        else:
                            lo = mid
                    ok.append((npb, hi))
                    break
                lo = R
    if fixed:
        nprobe, R = points[0]
    elif ok:
        qq = {pt: quick_qps(*pt) for pt in ok}
        nprobe, R = max(ok, key=lambda pt: qq[pt])
        log(f"[{role}] choose " + ", ".join(f"{pt}: {q:.0f} q/s" for pt, q in qq.items()))
    else:
        nprobe, R = max(rec, key=lambda pt: rec[pt])
        log(f"[{role}] no point reached recall 0.95; timing the best one {(nprobe, R)}")

    # the autotuner picks the launch choices of each timed shape (results are
    # unchanged by construction and checked by the library)
    tuned = {}
    cache = f"{args.tune_cache}.{role}" if args.tune_cache else ""
    loaded = idx.tune_load(cache) if cache and os.path.exists(cache) else 0
    if loaded:
        log(f"[{role}] {loaded} tuned shapes loaded from {cache}")
        tuned = {"loaded_from_cache": loaded}
    elif not args.no_autotune:
        for pt in ([(p, w.rerank_n) for p in w.nprobe] if not fixed else []) + [(nprobe, R)]:
            t_ = time.perf_counter()
            tuned[f"nprobe={pt[0]},rerank={pt[1]}"] = idx.autotune(Qb[0], pt[0], w.k, pt[1])
            log(f"[{role}] autotune {pt} ({time.perf_counter() - t_:.0f}s): "
                f"{tuned[f'nprobe={pt[0]},rerank={pt[1]}']}")
        if cache:
            idx.tune_save(cache)
    listed_qps = {f"{p}": quick_qps(p, w.rerank_n) for p in w.nprobe} if not fixed else {}
    # host re-rank: the batch's split into sub-batches (overlap of host and GPU
    # against fuller list-major items), each split tuned for its sub-batch size
    parts_qps = {}
    hp_used = None  # host sub-batches per batch (-1: the library's rule)
    if host_vectors and args.host_parts < 0:
        for p in (1, 2, 4):
            idx.set_option("host_parts", p)
            if not loaded and not args.no_autotune:
                t_ = time.perf_counter()
                r_ = idx.autotune(Qb[0], nprobe, w.k, R)
                log(f"[{role}] {p} host sub-batch(es): autotuned in {time.perf_counter() - t_:.0f}s, "
                    f"{r_['ms']:.2f} ms per sub-batch (built-in rule {r_['ms_default']:.2f}): {r_}")
            # batches in flight: the given number, else two and three
            for c in ([conc] if args.concurrency > 0 else [2, 3]):
                parts_qps[f"{p}@{c}"] = quick_qps(nprobe, R, steps=12, threads=c)
                log(f"[{role}] {p} host sub-batch(es), {c} in flight: {parts_qps[f'{p}@{c}']:.0f} q/s")
        best_key = max(parts_qps, key=parts_qps.get)
        best, conc = (int(x) for x in best_key.split("@"))
        idx.set_option("host_parts", best)
        hp_used = best
        log(f"[{role}] host sub-batches @ batches in flight: "
            + ", ".join(f"{k}: {q:.0f} q/s" for k, q in parts_qps.items()) + f"; using {best_key}")
        if cache and not loaded:
            idx.tune_save(cache)
    elif host_vectors:
        idx.set_option("host_parts", args.host_parts)
        hp_used = args.host_parts

    idx.set_option("scan", {"auto": 0, "popcount": 1, "mfma": 2}[args.scan])
    ids = torch.empty((w.nq, w.k), dtype=torch.int64, device=dev)
    dd = torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)
    nst = args.streams if args.streams > 0 else (1 if host_vectors else 2)
    streams_qps = {}
    if args.streams <= 0 and not host_vectors:
        # device-resident batches: two or three in flight from this thread
        # (the faster is timed)
        streams_qps = {str(n_): alternating_qps(idx, Qb, nprobe, w.k, R, n_, 12) for n_ in (2, 3)}
        nst = int(max(streams_qps, key=streams_qps.get))
        log(f"[{role}] streams: " + ", ".join(f"{k_}: {v_:.0f} q/s" for k_, v_ in streams_qps.items())
            + f"; using {nst}")
    streams = [torch.cuda.Stream(device=dev) for _ in range(nst)]
    outs = [(torch.empty((w.nq, w.k), dtype=torch.int64, device=dev),
             torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)) for _ in range(nst)]

    def step(s):
        st = streams[s % nst]
        oi, od = outs[s % nst]
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=oi, dists=od, stream=st.cuda_stream)

    steps = args.steps if role == "headline" else args.secondary_steps
    conc = min(conc, nst) if nst > 1 else conc
    if conc > 1 and nst < conc:
        streams += [torch.cuda.Stream(device=dev) for _ in range(conc - nst)]
        outs += [(torch.empty((w.nq, w.k), dtype=torch.int64, device=dev),
                  torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)) for _ in range(conc - nst)]
        nst = conc

    def run_steps(first, count):
        if conc == 1:
            for s in range(first, first + count):
                step(s)
            return
        import threading

        def worker(t):
            torch.cuda.set_device(dev)
            for s in range(first + t, first + count, conc):
                step(s)
        th = [threading.Thread(target=worker, args=(t,)) for t in range(conc)]
        for x in th:
            x.start()
        for x in th:
            x.join()

    torch.cuda.synchronize()
    run_steps(0, max(args.warmup, conc))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(0, steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = elapsed * 1e3 / steps
    qps = w.nq * steps / elapsed
    log(f"[{role}] timed {steps} steps ({conc} in flight): {qps:.0f} queries/s, {ms_step:.3f} ms per batch")
    # stage times, scanned work and per-launch kernel times: the same searches
    # again with the library's instrumentation on (kept out of the timed steps)
    idx.set_timing(True)
    for s in range(min(steps, 10)):
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=ids, dists=dd)
    torch.cuda.synchronize()
    tm = idx.timings()
    idx.set_timing(False)

    lat = []
    for s in range(args.latency_iters):
        torch.cuda.synchronize()
        t = time.perf_counter()
        idx.search(Qb[s % nb], nprobe, w.k, R, ids=ids, dists=dd)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    p50, p99 = float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # the scan forms at the chosen point (the in-house ablation of the work
    # schedule and of fused versus separate selection)
    variants = {}
    if not args.no_variants:
        for name, mode in (("tuned", 0), ("query_list_items_popcount_then_merge", 1),
                           ("list_major_work_queue", 2), ("one_item_per_query_fused_select", 3)):
            idx.set_option("scan", mode)
            variants[name] = quick_qps(nprobe, R, steps=6)
        idx.set_option("scan", 0)
        log(f"[{role}] scan forms: " + ", ".join(f"{k_}: {v:.0f} q/s" for k_, v in variants.items()))

    # the same lists under the other estimators: the unquantised query (the
    # paper's own precision point) and IVF-Flat (its comparison system), each
    # at the smallest re-rank list / probe count reaching recall 0.95
    estimators = {}
    if not args.no_estimators:
        grid = sorted({min(3840, f * w.rerank_n) for f in (1, 2, 3, 4, 5, 7, 10, 15, 20, 40)})
        if w.d <= 1024:
            idx.set_option("estimator", 1)
            row = {"nprobe": nprobe, "points": {}}
            for R1 in grid:
                r1 = eval_point(nprobe, R1)
                row["points"][str(R1)] = r1
                if r1 >= 0.95:
                    row.update(rerank_n=R1, recall_at_10=r1, qps=quick_qps(nprobe, R1, steps=4))
                    break
            estimators["unquantised_fp32_query"] = row
            log(f"[{role}] unquantised query at nprobe {nprobe}: {row}")
        if info["device_bytes"] and not args.no_flat and w.d <= 256:
            idx.set_option("estimator", 2)
            row = {"rerank_n": w.k, "points": {}}
            top = min(w.nlist, 4096)
            for npb in sorted({p for p in list(w.nprobe) + [256, 512, 1024, 2048] if p <= top}):
                rf = eval_point(npb, w.k)
                row["points"][str(npb)] = rf
                if rf >= 0.95:
                    row.update(nprobe=npb, recall_at_10=rf, qps=quick_qps(npb, w.k, steps=4))
                    break
            row["flat_bytes"] = (w.d + 3) // 4 * 4 * 4 * w.n + 4 * w.n
            if "qps" in row:
                row["rabitq_speedup_at_equal_recall"] = qps / row["qps"]
            estimators["ivf_flat"] = row
            log(f"[{role}] IVF-Flat: {row}")
        idx.set_option("estimator", 0)

    ns = max(1, tm["searches"])
    wname = w.name if w.n == get(w.name).n else f"{w.name}/n={w.n}"
    roofline = roofline_of(tm, w, wname, nprobe, R, args.scan)
    cpu = cpu_pool.run(nprobe, w.k, R) if cpu_pool else None
    out = {
        "value": qps, "ms_per_step": ms_step, "steps": steps,
        "config": {"workload": wname, "n": w.n, "d": w.d, "nlist": w.nlist, "nprobe": nprobe,
                   "batch": w.nq, "k": w.k, "rerank_n": R, "bq": w.bq, "rotation": args.rotation,
                   "rerank_on": "host" if host_vectors else "gpu",
                   "host_parts": hp_used,
                   "raw_vectors": "host (2 MiB pages), borrowed" if host_vectors else "HBM",
                   "streams": nst, "batches_in_flight": conc, "parallelism": "none (1 GPU)"},
        "recall_at_10": rec[(nprobe, R)], "recall_queries": gt_n,
        "recall_by_point": {f"nprobe={p},rerank={r}": v for (p, r), v in rec.items()},
        "probe_recall_by_nprobe": {str(p): v for p, v in prec.items()},
        "qps_at_listed_nprobe": listed_qps, "qps_by_scan_form": variants, "autotune": tuned,
        "qps_by_host_parts": parts_qps, "qps_by_streams": streams_qps,
        # queries whose list-major pool overflowed and were searched again
        "redo_queries_per_batch": tm["redo_queries"] / max(1, tm["searches"]),
        "p50_ms": p50, "p99_ms": p99,
        "stage_ms": {s: tm[f"{s}_ms"] / ns for s in
                     ("probe", "rotate", "quant", "scan", "merge", "rerank", "total")},
        "roofline": roofline, "estimators": estimators, "cpu_baseline": cpu, "gen_s": gen_s,
        "build_s": build_s,
        "index_info": info,
    }
    out["_gt"] = gt
    return idx, X, Qall, out, (nprobe, R)


def hbm_placement(w, X, Qall, parts, gt, nprobe, R, args):
    """The headline index with its raw vectors in HBM instead (GPU gather
    re-rank), from the same centroids, rotation and lists, at the same point.
    One MI355X holds the whole 400M x 96 set (154 GB of rows plus 8 GB of
    codes) in its 288 GB, so this is the placement the library's automatic
    rule would choose there."""
    import torch
    from paper_2605_16007_amd import Index
    dev = torch.device("cuda:0")
    t = time.perf_counter()
    ix = Index.build(X, w.nlist, bq=w.bq, centroids=parts["centroids"], rotation=parts["rotation"],
                     assignment=parts["assign"], vectors_on_host=False)
    build_s = time.perf_counter() - t
    try:
        free_b, _ = torch.cuda.mem_get_info()
        log(f"[headline] HBM placement built in {build_s:.0f}s ({ix.info()['device_bytes'] / 1e9:.1f} GB); "
            f"{free_b / 1e9:.1f} GB free")
        Qb = [torch.from_numpy(Qall[i * w.nq:(i + 1) * w.nq]).to(dev) for i in range(args.batches)]
        tuned = ix.autotune(Qb[0], nprobe, w.k, R) if not args.no_autotune else None
        free_b, _ = torch.cuda.mem_get_info()
        log(f"[headline] HBM placement tuned; {free_b / 1e9:.1f} GB free")
        # batches alternate over two or three streams from this thread, as in
        # the device-resident timing of measure()
        streams_qps = {}
        if args.streams > 0:
            nst = args.streams
        else:
            streams_qps = {str(n_): alternating_qps(ix, Qb, nprobe, w.k, R, n_, 8) for n_ in (2, 3)}
            nst = int(max(streams_qps, key=streams_qps.get))
        sts = [torch.cuda.Stream(device=dev) for _ in range(nst)]
        outs = [(torch.empty((w.nq, w.k), dtype=torch.int64, device=dev),
                 torch.empty((w.nq, w.k), dtype=torch.float32, device=dev)) for _ in range(nst)]

        def step(s):
            ix.search(Qb[s % len(Qb)], nprobe, w.k, R, ids=outs[s % nst][0], dists=outs[s % nst][1],
                      stream=sts[s % nst].cuda_stream)
        for s in range(max(args.warmup, nst)):
            step(s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            step(s)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r_ids, _ = ix.search(Qb[0], nprobe, w.k, R)
        torch.cuda.synchronize()
        rec = recall(r_ids[:len(gt)].cpu().numpy(), gt)
        out = {"qps": w.nq * args.steps / el, "ms_per_step": el * 1e3 / args.steps,
               "recall_at_10": rec, "nprobe": nprobe, "rerank_n": R, "rerank_on": "gpu",
               "raw_vectors": "HBM", "device_bytes": ix.info()["device_bytes"], "build_s": build_s,
               "streams": nst, "qps_by_streams": streams_qps,
               "autotune": tuned}
    finally:
        ix.close()
    log(f"[headline] vectors in HBM: {out['qps']:.0f} q/s at recall {out['recall_at_10']:.4f}")
    return out


def rerank_ablation(w, X, Qall, dev_idx, args):
    """GPU versus host re-rank at one probe count over several rerank_n: the
    same lists, once with the raw vectors in HBM (gather kernel) and once in
    huge-page host memory (host cores, overlapped with the GPU search)."""
    import torch
    from paper_2605_16007_amd import Index, huge_page_rows
    xt = huge_page_rows(*X.shape)
    xt[:] = X
    c = dev_idx.export("centroids")
    a = dev_idx.export("assign")
    P = dev_idx.export("rotation")
    host = Index.build(xt, w.nlist, bq=w.bq, centroids=c, rotation=P, assignment=a,
                       vectors_on_host=True, borrow_vectors=True)
    q = torch.from_numpy(Qall[:w.nq]).cuda()
    out = {}
    try:
        for R in (100, 200, 500, 1000):
            row = {}
            for name, ix in (("gpu", dev_idx), ("host", host)):
                ix.search(q, args.ablation_nprobe, w.k, R)
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(5):
                    ix.search(q, args.ablation_nprobe, w.k, R)
                torch.cuda.synchronize()
                row[name] = w.nq * 5 / (time.perf_counter() - t)
            out[str(R)] = row
            log(f"[ablation] rerank {R} at nprobe {args.ablation_nprobe}: GPU {row['gpu']:.0f} q/s, "
                f"host {row['host']:.0f} q/s")
    finally:
        host.close()
    return {"nprobe": args.ablation_nprobe, "qps_by_rerank_n": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--streams", type=int, default=0,
                    help="HIP streams the timed batches alternate over from one caller thread (each "
                         "batch whole on one); 0: two or three (the faster) when the raw vectors are "
                         "in HBM, else one")
    ap.add_argument("--workload", default="unit96_400m")
    ap.add_argument("--shard", action="store_true",
                    help="the 400M-row workload's first 50M rows (nlist 8192) instead of the whole set")
    ap.add_argument("--n", type=int, default=0, help="database rows (nlist scales with them)")
    ap.add_argument("--vectors-on-device", action="store_true",
                    help="keep the raw vectors in HBM even where the workload puts them on the host")
    ap.add_argument("--nprobe", type=int, default=0,
                    help="fix nprobe (default: the fastest point reaching recall@10 >= 0.95)")
    ap.add_argument("--rerank", type=int, default=0, help="fix rerank_n (with --nprobe)")
    ap.add_argument("--batches", type=int, default=4, help="distinct query batches cycled")
    ap.add_argument("--gt-queries", type=int, default=0,
                    help="queries with exact kNN for recall (default: the batch; 1000 above 100M rows)")
    ap.add_argument("--latency-iters", type=int, default=30)
    ap.add_argument("--kmeans-iters", type=int, default=0)
    ap.add_argument("--kmeans-restarts", type=int, default=0)
    ap.add_argument("--train-n", type=int, default=0)
    ap.add_argument("--kmeans-init", choices=("kmeans++", "random"), default="",
                    help="initial centroids of the library's k-means (default: its own, k-means++)")
    ap.add_argument("--cpu-queries", type=int, default=128)
    ap.add_argument("--cpu-cores", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rotation", choices=("fp32", "bf16"), default="fp32")
    ap.add_argument("--no-autotune", action="store_true", help="time the built-in launch rule")
    ap.add_argument("--tune-cache", default="",
                    help="autotune cache prefix: <prefix>.<role> is loaded if it exists, else written")
    ap.add_argument("--no-variants", action="store_true", help="skip the scan-form ablation")
    ap.add_argument("--no-estimators", action="store_true",
                    help="skip the unquantised-query and IVF-Flat comparisons")
    ap.add_argument("--no-flat", action="store_true", help="build no IVF-Flat copy of the lists")
    ap.add_argument("--concurrency", type=int, default=0,
                    help="batches in flight from as many caller threads (default: with the "
                         "re-rank on host cores the faster of 2 and 3 in a short trial, else 1 "
                         "caller thread over --streams)")
    ap.add_argument("--host-parts", type=int, default=-1,
                    help="sub-batches of a host re-rank search (0: the library's rule; default: "
                         "the fastest of 1, 2 and 4, each autotuned)")
    ap.add_argument("--no-hbm-variant", action="store_true",
                    help="skip timing the host-vector headline with its vectors in HBM")
    ap.add_argument("--scan", choices=("auto", "popcount", "mfma"), default="auto",
                    help="force the scan form of the timed loop (auto: tuned per chunk)")
    ap.add_argument("--secondary", default="sift10m",
                    help="a second workload measured after the headline ('' skips it)")
    ap.add_argument("--secondary-steps", type=int, default=20)
    ap.add_argument("--others", default="mixture128,embed960",
                    help="further workloads measured briefly (comma-separated; empty: none)")
    ap.add_argument("--ablation-nprobe", type=int, default=512,
                    help="probe count of the GPU-versus-host re-rank ablation on the secondary workload")
    ap.add_argument("--serve-rates", default="5000,10000,20000,50000",
                    help="Poisson arrival rates (queries/s) of the serving comparison on the "
                         "secondary workload's index ('' skips it)")
    ap.add_argument("--serve-seconds", type=float, default=1.0, help="seconds of arrivals per rate")
    ap.add_argument("--serve-max", type=int, default=20000, help="most requests per rate")
    ap.add_argument("--serve-warmup-s", type=float, default=0.2,
                    help="seconds of arrivals served before each rate's measured trace")
    ap.add_argument("--plain-max", type=int, default=3000,
                    help="most requests of each trace replayed one query at a time")
    ap.add_argument("--calibrate-copy-gib", type=float, default=0.0,
                    help="finish with one device-to-device copy of this size (PMC calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures the search path on one GPU only; this build runs no "
              "multi-GPU configuration (--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    from synth import get, queries
    w = get(args.workload)
    shard_note = None
    n = args.n or (SHARD_ROWS if (w.name == "unit96_400m" and args.shard) else 0)
    if n and n != w.n:
        w = w.with_(n=n, nlist=max(1, int(round(w.nlist * n / w.n))))
        if w.name == "unit96_400m":
            shard_note = True
    big = w.n > 100_000_000
    given = {k_: getattr(args, k_) for k_ in ("kmeans_init", "kmeans_iters", "kmeans_restarts", "no_flat")}
    if big:
        # the whole set: random initial centroids, 10 iterations, one run
        # (options given on the command line win); no IVF-Flat copy (its 155 GB
        # and the build's staged rows would not fit in HBM together)
        args.kmeans_init = args.kmeans_init or "random"
        args.kmeans_iters = args.kmeans_iters or 10
        args.kmeans_restarts = args.kmeans_restarts or 1
        args.no_flat = True
    user_gt = args.gt_queries
    if not args.gt_queries:
        args.gt_queries = 1000 if big else 10_000
    host_vectors = w.kind == "unit_mixture" and not args.vectors_on_device

    cpu_pool = None
    if not args.no_cpu_baseline:
        # forked before the GPU is touched
        cores = args.cpu_cores or min(16, os.cpu_count() or 1)
        cpu_pool = CpuBaseline(w, queries(w, w.nq), args.cpu_queries, cores)

    import torch
    torch.cuda.set_device(0)
    idx, X, Qall, head, (nprobe, R) = measure(w, args, host_vectors=host_vectors, role="headline",
                                              cpu_pool=cpu_pool)
    gt = head.pop("_gt")
    if cpu_pool:
        cpu_pool.close()
    hbm_parts = None
    if host_vectors and not args.no_hbm_variant:
        # (the host-vector index and its workspaces are freed first: the whole
        # set's rows then fill 154 GB of HBM)
        hbm_parts = {what: idx.export(what) for what in ("centroids", "rotation", "assign")}
    if shard_note:
        import psutil
        full = get("unit96_400m")
        ram = psutil.virtual_memory().total
        head["shard"] = {
            "of": f"{full.name}: {full.n} x {full.d}, nlist {full.nlist}",
            "rows": w.n, "nlist": w.nlist, "host_ram_bytes": ram,
            "full_raw_vector_bytes": full.n * full.d * 4,
            "shard_build_s": head["build_s"],
            "reason": (f"--shard: the first {w.n} rows with nlist {w.nlist} keep the lists' length "
                       f"({w.n // w.nlist} vectors on average) and the batch shape, but each list is "
                       f"probed by {full.nlist // w.nlist}x more of a batch's queries than in the "
                       f"whole set, so list-major items are fuller than there"),
        }
        log(f"[headline] shard: {head['shard']['reason']}")
    idx.close()
    if hbm_parts is not None:
        from paper_2605_16007_amd import RbqError
        torch.cuda.empty_cache()
        free_b, total_b = torch.cuda.mem_get_info()
        log(f"[headline] device memory before the HBM placement: {free_b / 1e9:.1f} GB free of "
            f"{total_b / 1e9:.1f} GB (torch holds {torch.cuda.memory_reserved() / 1e9:.1f} GB)")
        try:
            head["vectors_in_hbm"] = hbm_placement(w, X, Qall, hbm_parts, gt, nprobe, R, args)
        except RbqError as e:
            free_b, _ = torch.cuda.mem_get_info()
            log(f"[headline] HBM placement failed ({e}); {free_b / 1e9:.1f} GB free")
            head["vectors_in_hbm"] = {"error": str(e)}
        hbm_parts = None
    del X

    secondary = None
    if args.secondary:
        w2 = get(args.secondary)
        sargs = argparse.Namespace(**vars(args))
        sargs.nprobe = 0
        sargs.rerank = 0
        sargs.gt_queries = min(user_gt or w2.nq, w2.nq)
        for k_, v in given.items():  # the whole set's build choices are its own
            setattr(sargs, k_, v)
        hint = [(512, 3840)] if w2.name == "sift10m" else None
        idx2, X2, Q2, sec, _ = measure(w2, sargs, host_vectors=False, role="secondary", points_hint=hint)
        sec.pop("_gt")
        if args.ablation_nprobe and w2.kind != "unit_mixture":
            sec["rerank_ablation"] = rerank_ablation(w2, X2, Q2, idx2, args)
        if args.serve_rates:
            sec["serving"] = serve_compare(idx2, w2, args)
        secondary = sec
        idx2.close()

    # the remaining workloads, briefly: the small mixture (the paper's plain
    # IVF-RaBitQ configuration) and the 960-dimension features with FP32
    # against BF16 query rotation
    others = {}
    for name in [x for x in args.others.split(",") if x]:
        w3 = get(name)
        oargs = argparse.Namespace(**vars(args))
        oargs.nprobe = oargs.rerank = 0
        oargs.gt_queries = w3.nq
        oargs.no_variants = oargs.no_estimators = True
        oargs.no_flat = True
        oargs.cpu_queries = 0
        for k_, v in given.items():
            setattr(oargs, k_, v)
        oargs.no_flat = True
        idx3, X3, Q3, o3, (np3, R3) = measure(w3, oargs, host_vectors=False, role=name)
        gt3 = o3.pop("_gt")
        row = {k_: o3[k_] for k_ in ("value", "ms_per_step", "recall_at_10", "recall_by_point",
                                     "p50_ms", "p99_ms", "build_s")}
        row["config"] = o3["config"]
        if w3.d >= 512:
            # BF16 inputs to the query rotation (FP32 accumulation) at the same point
            idx3.set_option("rotation", 1)
            q3 = torch.from_numpy(Q3[:w3.nq]).cuda()
            ids3, _ = idx3.search(q3, np3, w3.k, R3)
            torch.cuda.synchronize()
            rb = recall(ids3[:len(gt3)].cpu().numpy(), gt3)
            t_ = time.perf_counter()
            for _ in range(10):
                idx3.search(q3, np3, w3.k, R3)
            torch.cuda.synchronize()
            row["bf16_rotation"] = {"recall_at_10": rb, "qps": w3.nq * 10 / (time.perf_counter() - t_)}
            idx3.set_option("rotation", 0)
            log(f"[{name}] BF16 rotation: recall {rb:.4f}, {row['bf16_rotation']['qps']:.0f} q/s")
        others[name] = row
        idx3.close()
        del X3

    if args.calibrate_copy_gib > 0:
        nbytes = int(args.calibrate_copy_gib * (1 << 30)) // 4
        a = torch.ones(nbytes, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[calibrate] copied {nbytes * 4} bytes device to device")
        del a, b

    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": head["steps"],
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
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
    }
    line.update({k_: v for k_, v in head.items() if k_ not in ("value", "ms_per_step", "steps")})
    line["secondary"] = secondary
    line["other_workloads"] = others
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
