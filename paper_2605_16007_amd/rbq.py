"""Python binding of librbq (ctypes). Argument marshalling only: every step of
index construction and search runs in the library's HIP kernels.

Arrays may be NumPy (host) or torch tensors (host or GPU); torch is used for
device memory and streams only. The library must be built
(``python -m paper_2605_16007_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbq.so")

RBQ_OK, RBQ_EINVAL, RBQ_ENOMEM, RBQ_EDEVICE, RBQ_ESTATE, RBQ_EAGAIN = 0, -1, -2, -3, -4, -5
EXPORT = {"centroids": 1, "rotation": 2, "assign": 3, "codes": 4, "factors": 5, "list_sizes": 6}

# every symbol declared in include/rbq.h
SYMBOLS = [
    "rbq_build_params_init", "rbq_build_index", "rbq_free_index", "rbq_get_info", "rbq_search",
    "rbq_export", "rbq_search_debug", "rbq_set_timing", "rbq_get_timings", "rbq_save",
    "rbq_load", "rbq_last_error", "rbq_version", "rbq_set_option", "rbq_search_mixed",
    "rbq_server_params_init", "rbq_server_create", "rbq_submit", "rbq_poll", "rbq_wait",
    "rbq_server_get_stats", "rbq_server_destroy", "rbq_server_replay", "rbq_replay_plain",
    "rbq_autotune", "rbq_tune_save", "rbq_tune_load", "rbq_tune_clear", "rbq_search_noalloc",
]
OPTIONS = {"scan": 1, "group_min": 2, "pool_cap": 3, "rotation": 4, "group_size": 5, "estimator": 6,
           "block": 7, "host_parts": 8}


class BuildParams(C.Structure):
    _fields_ = [("nlist", C.c_int32), ("bq", C.c_int32), ("seed", C.c_uint64),
                ("kmeans_iters", C.c_int32), ("kmeans_restarts", C.c_int32),
                ("train_n", C.c_int64), ("rotation", C.c_void_p), ("centroids", C.c_void_p),
                ("assignment", C.c_void_p), ("vectors_on_host", C.c_int32),
                ("host_threads", C.c_int32), ("borrow_vectors", C.c_int32),
                ("ivf_flat", C.c_int32), ("kmeans_init", C.c_int32), ("reserved", C.c_int32 * 3)]


class IndexInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("nlist", C.c_int32), ("bq", C.c_int32),
                ("vectors_on_host", C.c_int32), ("max_list_len", C.c_int64),
                ("device_bytes", C.c_int64), ("code_bytes", C.c_int64),
                ("vectors_borrowed", C.c_int32), ("reserved", C.c_int32)]


class DebugIO(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "inject_probes", "inject_qu", "inject_scalars", "probes", "probe_score", "qrot", "qu",
        "scalars", "ip", "est", "cand_ids", "cand_est", "ids", "sqdist")] + [
        ("probe_chunk", C.c_int32), ("reserved", C.c_int32), ("inject_qrot", C.c_void_p)]


class Timings(C.Structure):
    _fields_ = [("searches", C.c_int64), ("probe_ms", C.c_float), ("rotate_ms", C.c_float),
                ("quant_ms", C.c_float), ("scan_ms", C.c_float), ("merge_ms", C.c_float),
                ("rerank_ms", C.c_float), ("total_ms", C.c_float),
                ("scanned_vectors", C.c_int64), ("scan_bytes", C.c_int64),
                ("read_bytes", C.c_int64), ("group_launches", C.c_int64),
                ("popc_launches", C.c_int64), ("group_scan_ms", C.c_float),
                ("group_vectors", C.c_int64), ("group_read_bytes", C.c_int64),
                ("fused_launches", C.c_int64), ("fused_scan_ms", C.c_float),
                ("reserved", C.c_int32), ("fused_vectors", C.c_int64),
                ("fused_read_bytes", C.c_int64), ("redo_queries", C.c_int64)]


class ServerParams(C.Structure):
    _fields_ = [("lanes", C.c_int32), ("max_batch", C.c_int32), ("queue_cap", C.c_int32),
                ("max_nprobe", C.c_int32), ("max_k", C.c_int32), ("max_rerank", C.c_int32),
                ("mem_budget", C.c_int64), ("reserved", C.c_int32 * 8)]


class ServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("rejected", C.c_int64), ("completed", C.c_int64),
                ("batches", C.c_int64), ("max_batch_seen", C.c_int64),
                ("budget_cuts", C.c_int64), ("reserved", C.c_int64 * 2)]


class ReplayIO(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "q", "nprobe", "k", "rerank_n", "arrival_s", "ids", "sqdist", "latency_s")] + [
        ("n", C.c_int64), ("k_stride", C.c_int32), ("reserved", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("scan", C.c_int32), ("group_size", C.c_int32), ("wg_per_cu", C.c_int32),
                ("first_factor", C.c_int32), ("ms", C.c_float), ("ms_default", C.c_float),
                ("trials", C.c_int32), ("chunk_group_min", C.c_int32),
                ("growth", C.c_int32), ("early_form", C.c_int32), ("block", C.c_int32),
                ("merge_form", C.c_int32)]


class RbqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librbq status {status}: {msg}")
        self.status = status


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_16007_amd.build`")
        # torch ships its own HIP runtime under the same soname; load it first
        # so that librbq and torch share one runtime in this process
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        L.rbq_build_params_init.argtypes = [C.POINTER(BuildParams)]
        L.rbq_build_params_init.restype = None
        L.rbq_build_index.argtypes = [vp, i64, i32, C.POINTER(BuildParams), C.POINTER(vp)]
        L.rbq_free_index.argtypes = [vp]
        L.rbq_get_info.argtypes = [vp, C.POINTER(IndexInfo)]
        L.rbq_search.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, vp]
        L.rbq_search_noalloc.argtypes = [vp, vp, i64, i32, i32, i32, vp, vp, vp]
        L.rbq_export.argtypes = [vp, i32, vp, C.c_size_t]
        L.rbq_search_debug.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(DebugIO)]
        L.rbq_set_timing.argtypes = [vp, i32]
        L.rbq_get_timings.argtypes = [vp, C.POINTER(Timings)]
        L.rbq_set_option.argtypes = [vp, i32, i64]
        L.rbq_save.argtypes = [vp, C.c_char_p]
        L.rbq_load.argtypes = [C.c_char_p, C.POINTER(vp)]
        L.rbq_last_error.restype = C.c_char_p
        L.rbq_last_error.argtypes = []
        L.rbq_version.restype = C.c_char_p
        L.rbq_version.argtypes = []
        L.rbq_search_mixed.argtypes = [vp, vp, i64, vp, vp, vp, i32, vp, vp, vp]
        L.rbq_server_params_init.argtypes = [C.POINTER(ServerParams)]
        L.rbq_server_create.argtypes = [vp, C.POINTER(ServerParams), C.POINTER(vp)]
        L.rbq_submit.argtypes = [vp, vp, i32, i32, i32, C.POINTER(C.c_uint64)]
        L.rbq_poll.argtypes = [vp, C.c_uint64, vp, vp, C.POINTER(i32), C.POINTER(i64)]
        L.rbq_wait.argtypes = [vp, C.c_uint64, vp, vp, i64, C.POINTER(i64)]
        L.rbq_server_get_stats.argtypes = [vp, C.POINTER(ServerStats)]
        L.rbq_server_destroy.argtypes = [vp]
        L.rbq_server_replay.argtypes = [vp, C.POINTER(ReplayIO)]
        L.rbq_replay_plain.argtypes = [vp, C.POINTER(ReplayIO)]
        L.rbq_autotune.argtypes = [vp, vp, i64, i32, i32, i32, C.POINTER(TuneResult)]
        L.rbq_tune_save.argtypes = [vp, C.c_char_p]
        L.rbq_tune_load.argtypes = [vp, C.c_char_p, C.POINTER(i32)]
        L.rbq_tune_clear.argtypes = [vp]
        for name in SYMBOLS:
            if name not in ("rbq_build_params_init", "rbq_last_error", "rbq_version"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(status):
    if status != RBQ_OK:
        raise RbqError(status, lib().rbq_last_error().decode())


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def _ptr(a):
    """Address of a contiguous NumPy array or torch tensor (None -> NULL)."""
    if a is None:
        return None
    if _is_torch(a):
        assert a.is_contiguous(), "tensor must be contiguous"
        return a.data_ptr()
    assert isinstance(a, np.ndarray) and a.flags.c_contiguous, "array must be C-contiguous"
    return a.ctypes.data


def _stream_of(t, stream):
    if stream is not None:
        return stream
    if _is_torch(t) and t.is_cuda:
        import torch
        return torch.cuda.current_stream(t.device).cuda_stream
    return None


class Index:
    """An IVF-RaBitQ index held by librbq on the current GPU."""

    def __init__(self, handle):
        self._h = C.c_void_p(handle)

    # ---------------------------------------------------------------- build
    @classmethod
    def build(cls, x, nlist, *, bq=4, seed=0, kmeans_iters=25, kmeans_restarts=3, train_n=0,
              rotation=None, centroids=None, assignment=None, vectors_on_host=None,
              host_threads=0, borrow_vectors=False, ivf_flat=False, kmeans_init="kmeans++"):
        """Build an index over x (NumPy array or torch tensor, n x d float32).
        vectors_on_host: False (HBM), True (host memory, host re-rank) or None
        (automatic). borrow_vectors: keep x itself (host memory, pageable or
        pinned; rows backed by huge pages, see ``huge_page_rows``, re-rank
        fastest) as the host rows; the caller keeps it alive and unchanged while
        the index exists."""
        if _is_torch(x):
            assert str(x.dtype) == "torch.float32"
        else:
            x = np.ascontiguousarray(x, np.float32)
        n, d = x.shape
        p = BuildParams()
        lib().rbq_build_params_init(C.byref(p))
        p.nlist, p.bq, p.seed = int(nlist), int(bq), int(seed)
        p.kmeans_iters, p.kmeans_restarts, p.train_n = int(kmeans_iters), int(kmeans_restarts), int(train_n)
        keep = []
        if rotation is not None:
            rotation = np.ascontiguousarray(rotation, np.float32)
            keep.append(rotation)
            p.rotation = rotation.ctypes.data
        if centroids is not None:
            centroids = np.ascontiguousarray(centroids, np.float32)
            keep.append(centroids)
            p.centroids = centroids.ctypes.data
        if assignment is not None:
            assignment = np.ascontiguousarray(assignment, np.int32)
            keep.append(assignment)
            p.assignment = assignment.ctypes.data
        p.vectors_on_host = -1 if vectors_on_host is None else int(bool(vectors_on_host))
        p.host_threads = int(host_threads)
        p.borrow_vectors = int(bool(borrow_vectors))
        p.ivf_flat = int(bool(ivf_flat))
        p.kmeans_init = {"kmeans++": 0, "random": 1}[kmeans_init]
        h = C.c_void_p()
        _check(lib().rbq_build_index(_ptr(x), n, d, C.byref(p), C.byref(h)))
        ix = cls(h.value)
        if borrow_vectors:
            ix._borrowed = x  # the index reads these rows until it is freed
        return ix

    @classmethod
    def load(cls, path):
        h = C.c_void_p()
        _check(lib().rbq_load(os.fsencode(path), C.byref(h)))
        return cls(h.value)

    def save(self, path):
        _check(lib().rbq_save(self._h, os.fsencode(path)))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().rbq_free_index(self._h))
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- info / export
    def info(self) -> dict:
        i = IndexInfo()
        _check(lib().rbq_get_info(self._h, C.byref(i)))
        return {f: getattr(i, f) for f, _ in IndexInfo._fields_}

    def export(self, what: str) -> np.ndarray:
        inf = self.info()
        n, d, nlist = inf["n"], inf["d"], inf["nlist"]
        shape, dt = {
            "centroids": ((nlist, d), np.float32), "rotation": ((d, d), np.float32),
            "assign": ((n,), np.int32), "codes": ((n, (d + 7) // 8), np.uint8),
            "factors": ((n, 2), np.float32), "list_sizes": ((nlist,), np.int64),
        }[what]
        out = np.empty(shape, dt)
        _check(lib().rbq_export(self._h, EXPORT[what], out.ctypes.data, out.nbytes))
        return out

    # ---------------------------------------------------------------- search
    def search(self, q, nprobe, k, rerank_n, ids=None, dists=None, stream=None):
        """Top-k (ids int64, squared distances float32) per query. With a GPU
        tensor ``q`` the outputs are GPU tensors on the caller's stream."""
        if _is_torch(q):
            import torch
            nq = q.shape[0]
            if ids is None:
                ids = torch.empty((nq, k), dtype=torch.int64, device=q.device)
            if dists is None:
                dists = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        else:
            q = np.ascontiguousarray(q, np.float32)
            nq = q.shape[0]
            if ids is None:
                ids = np.empty((nq, k), np.int64)
            if dists is None:
                dists = np.empty((nq, k), np.float32)
        s = _stream_of(q, stream)
        _check(lib().rbq_search(self._h, _ptr(q), nq, int(nprobe), int(k), int(rerank_n),
                                _ptr(ids), _ptr(dists), s))
        return ids, dists

    def search_noalloc(self, q, nprobe, k, rerank_n, ids=None, dists=None, stream=None):
        """rbq_search on the library's fixed per-GPU workspace (no device
        allocation): q, and ids / dists if given, are GPU tensors."""
        import torch
        nq = q.shape[0]
        if ids is None:
            ids = torch.empty((nq, k), dtype=torch.int64, device=q.device)
        if dists is None:
            dists = torch.empty((nq, k), dtype=torch.float32, device=q.device)
        s = _stream_of(q, stream)
        _check(lib().rbq_search_noalloc(self._h, _ptr(q), nq, int(nprobe), int(k), int(rerank_n),
                                        _ptr(ids), _ptr(dists), s))
        return ids, dists

    def search_mixed(self, q, nprobe, k, rerank_n, stream=None):
        """Mixed batch: query i with its own nprobe[i], k[i], rerank_n[i]. Returns
        (ids, dists) of shape (nq, max k); row i is padded with (-1, inf) past
        k[i]. Outputs follow ``q`` (NumPy or torch on q's device)."""
        nq = q.shape[0]
        nprobe = np.ascontiguousarray(np.broadcast_to(nprobe, (nq,)), np.int32)
        k = np.ascontiguousarray(np.broadcast_to(k, (nq,)), np.int32)
        rerank_n = np.ascontiguousarray(np.broadcast_to(rerank_n, (nq,)), np.int32)
        ks = int(k.max()) if nq else 1
        if _is_torch(q):
            import torch
            ids = torch.empty((nq, ks), dtype=torch.int64, device=q.device)
            dists = torch.empty((nq, ks), dtype=torch.float32, device=q.device)
        else:
            q = np.ascontiguousarray(q, np.float32)
            ids = np.empty((nq, ks), np.int64)
            dists = np.empty((nq, ks), np.float32)
        s = _stream_of(q, stream)
        _check(lib().rbq_search_mixed(self._h, _ptr(q), nq, nprobe.ctypes.data, k.ctypes.data,
                                      rerank_n.ctypes.data, ks, _ptr(ids), _ptr(dists), s))
        return ids, dists

    def replay_plain(self, q, nprobe, k, rerank_n, arrival_s):
        """Serve an open-loop trace one query at a time (rbq_search, nq = 1) in
        arrival order; returns (ids, dists, latency_s)."""
        return _replay(lambda io: lib().rbq_replay_plain(self._h, C.byref(io)),
                       q, nprobe, k, rerank_n, arrival_s)

    DEBUG_OUTPUTS = ("probes", "probe_score", "qrot", "qu", "scalars", "ip", "est", "cand_ids",
                     "cand_est", "ids", "sqdist")

    def search_debug(self, q, nprobe, k, rerank_n, *, inject_probes=None, inject_qu=None,
                     inject_scalars=None, inject_qrot=None, want=None, probe_chunk=0):
        """Stage-by-stage search (host arrays). Returns a dict of the stage
        outputs named in ``want`` (default: all); see rbq_search_debug in
        include/rbq.h for the layouts."""
        q = np.ascontiguousarray(q, np.float32)
        nq, d = q.shape
        want = set(self.DEBUG_OUTPUTS if want is None else want)
        maxlen = max(1, self.info()["max_list_len"]) if want & {"ip", "est"} else 1
        pairs = nq * nprobe
        out = {
            "probes": np.zeros((nq, nprobe), np.int32),
            "probe_score": np.zeros((nq, nprobe), np.float32),
            "qrot": np.zeros((nq, d), np.float32),
            "qu": np.zeros((nq, nprobe, d), np.uint8),
            "scalars": np.zeros((nq, nprobe, 4), np.float32),
            "ip": np.zeros((nq, nprobe, maxlen), np.int32),
            "est": np.zeros((nq, nprobe, maxlen), np.float32),
            "cand_ids": np.zeros((nq, rerank_n), np.int64),
            "cand_est": np.zeros((nq, rerank_n), np.float32),
            "ids": np.zeros((nq, k), np.int64),
            "sqdist": np.zeros((nq, k), np.float32),
        }
        out = {key: v for key, v in out.items() if key in want}
        io = DebugIO()
        keep = []
        if inject_probes is not None:
            a = np.ascontiguousarray(inject_probes, np.int32).reshape(pairs)
            keep.append(a)
            io.inject_probes = a.ctypes.data
            out.pop("probe_score", None)
        if inject_qu is not None:
            a = np.ascontiguousarray(inject_qu, np.uint8).reshape(pairs * d)
            b = np.ascontiguousarray(inject_scalars, np.float32).reshape(pairs * 3)
            keep += [a, b]
            io.inject_qu, io.inject_scalars = a.ctypes.data, b.ctypes.data
        if inject_qrot is not None:
            a = np.ascontiguousarray(inject_qrot, np.float32).reshape(nq * d)
            keep.append(a)
            io.inject_qrot = a.ctypes.data
        for key, arr in out.items():
            setattr(io, key, arr.ctypes.data)
        io.probe_chunk = int(probe_chunk)
        _check(lib().rbq_search_debug(self._h, q.ctypes.data, nq, int(nprobe), int(k),
                                      int(rerank_n), C.byref(io)))
        return out

    def autotune(self, q, nprobe, k, rerank_n) -> dict:
        """Time the result-preserving launch choices on these queries and keep
        the fastest for this batch shape (rbq_autotune)."""
        if not _is_torch(q):
            q = np.ascontiguousarray(q, np.float32)
        r = TuneResult()
        _check(lib().rbq_autotune(self._h, _ptr(q), q.shape[0], int(nprobe), int(k), int(rerank_n),
                                  C.byref(r)))
        return {f: getattr(r, f) for f, _ in TuneResult._fields_ if f != "reserved"}

    def tune_save(self, path):
        _check(lib().rbq_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path) -> int:
        n = C.c_int32()
        _check(lib().rbq_tune_load(self._h, os.fsencode(path), C.byref(n)))
        return n.value

    def tune_clear(self):
        _check(lib().rbq_tune_clear(self._h))

    def set_option(self, name: str, value: int):
        """Tuning knobs: scan (0 auto, 1 query-major popcount, 2 list-major
        MFMA, 3 one item per query), group_min, pool_cap, rotation,
        group_size, estimator (0 B_q-bit query, 1 unquantised, 2 IVF-Flat),
        block, host_parts; see rbq_set_option in include/rbq.h."""
        _check(lib().rbq_set_option(self._h, OPTIONS[name], int(value)))

    # ---------------------------------------------------------------- timing
    def set_timing(self, enabled: bool):
        _check(lib().rbq_set_timing(self._h, int(bool(enabled))))

    def timings(self) -> dict:
        t = Timings()
        _check(lib().rbq_get_timings(self._h, C.byref(t)))
        return {f: getattr(t, f) for f, _ in Timings._fields_}


def version() -> str:
    return lib().rbq_version().decode()


def huge_page_rows(n: int, d: int) -> np.ndarray:
    """An n x d float32 array in anonymous host memory, 2 MiB-aligned and
    advised for transparent huge pages: rows for an index that borrows its host
    vectors (the host re-rank gathers one random row per candidate, so 2 MiB
    pages cut its TLB misses). The array owns its mapping."""
    import mmap
    huge = 2 << 20
    nbytes = max(1, int(n) * int(d) * 4)
    length = -(-nbytes // huge) * huge
    # private, not the default shared mapping: shared anonymous memory is
    # shmem, whose huge pages are governed by another setting (often off)
    mm = mmap.mmap(-1, length + huge, flags=mmap.MAP_PRIVATE | mmap.MAP_ANONYMOUS)
    base = np.frombuffer(mm, np.uint8, count=1).ctypes.data
    off = (-base) % huge
    if hasattr(mmap, "MADV_HUGEPAGE"):
        mm.madvise(mmap.MADV_HUGEPAGE, off, length)
    return np.frombuffer(mm, np.float32, count=int(n) * int(d), offset=off).reshape(int(n), int(d))


def _replay(call, q, nprobe, k, rerank_n, arrival_s):
    q = np.ascontiguousarray(q, np.float32)
    n = q.shape[0]
    nprobe = np.ascontiguousarray(np.broadcast_to(nprobe, (n,)), np.int32)
    k = np.ascontiguousarray(np.broadcast_to(k, (n,)), np.int32)
    rerank_n = np.ascontiguousarray(np.broadcast_to(rerank_n, (n,)), np.int32)
    arrival_s = np.ascontiguousarray(arrival_s, np.float64)
    assert arrival_s.shape == (n,)
    ks = int(k.max()) if n else 1
    ids = np.empty((n, ks), np.int64)
    dists = np.empty((n, ks), np.float32)
    lat = np.empty(n, np.float64)
    io = ReplayIO()
    io.q, io.nprobe, io.k, io.rerank_n = q.ctypes.data, nprobe.ctypes.data, k.ctypes.data, rerank_n.ctypes.data
    io.arrival_s, io.ids, io.sqdist, io.latency_s = (arrival_s.ctypes.data, ids.ctypes.data,
                                                     dists.ctypes.data, lat.ctypes.data)
    io.n, io.k_stride = n, ks
    _check(call(io))
    return ids, dists, lat


class Server:
    """Continuous-batching serving loop over a resident index (rbq_server_*).
    The index must outlive the server."""

    def __init__(self, index: Index, *, lanes=2, max_batch=1024, queue_cap=65536, max_nprobe=0,
                 max_k=100, max_rerank=1000, mem_budget=1 << 30):
        p = ServerParams()
        _check(lib().rbq_server_params_init(C.byref(p)))
        p.lanes, p.max_batch, p.queue_cap = int(lanes), int(max_batch), int(queue_cap)
        p.max_nprobe, p.max_k, p.max_rerank = int(max_nprobe), int(max_k), int(max_rerank)
        p.mem_budget = int(mem_budget)
        h = C.c_void_p()
        _check(lib().rbq_server_create(index._h, C.byref(p), C.byref(h)))
        self._h = h
        self._index = index  # keeps the index alive

    def submit(self, q, nprobe, k, rerank_n):
        """Queue one query (host, d floats). Returns its ticket, or None when
        the queue is full (RBQ_EAGAIN)."""
        q = np.ascontiguousarray(q, np.float32).reshape(-1)
        t = C.c_uint64()
        st = lib().rbq_submit(self._h, q.ctypes.data, int(nprobe), int(k), int(rerank_n), C.byref(t))
        if st == RBQ_EAGAIN:
            return None
        _check(st)
        return t.value

    def poll(self, ticket, k):
        """(ids, dists, latency_ns) when finished, else None."""
        ids = np.empty(k, np.int64)
        dists = np.empty(k, np.float32)
        done = C.c_int32()
        lat = C.c_int64()
        _check(lib().rbq_poll(self._h, ticket, ids.ctypes.data, dists.ctypes.data, C.byref(done),
                              C.byref(lat)))
        return (ids, dists, lat.value) if done.value else None

    def wait(self, ticket, k, timeout_us=-1):
        """Block for the result; (ids, dists, latency_ns), or None on time-out."""
        ids = np.empty(k, np.int64)
        dists = np.empty(k, np.float32)
        lat = C.c_int64()
        st = lib().rbq_wait(self._h, ticket, ids.ctypes.data, dists.ctypes.data, int(timeout_us),
                            C.byref(lat))
        if st == RBQ_EAGAIN:
            return None
        _check(st)
        return ids, dists, lat.value

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().rbq_server_get_stats(self._h, C.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_ if f != "reserved"}

    def replay(self, q, nprobe, k, rerank_n, arrival_s):
        """Open-loop replay of an arrival trace through the server; returns
        (ids, dists, latency_s) with latency from each arrival time."""
        return _replay(lambda io: lib().rbq_server_replay(self._h, C.byref(io)),
                       q, nprobe, k, rerank_n, arrival_s)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _check(lib().rbq_server_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
