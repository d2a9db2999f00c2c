"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/rbq.h declares, and rejects bad arguments with RBQ_EINVAL before
touching a GPU (so these run on a machine without one)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2605_16007_amd import rbq

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "rbq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbq_[a-z_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(rbq.SYMBOLS)


def test_library_exports_every_symbol():
    L = rbq.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert "gfx950" in rbq.version()


def _params(**kw):
    p = rbq.BuildParams()
    rbq.lib().rbq_build_params_init(C.byref(p))
    p.nlist = 4
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_params_defaults():
    p = _params()
    assert p.bq == 4 and p.kmeans_iters == 25 and p.kmeans_restarts == 3 and p.train_n == 0
    assert p.vectors_on_host == -1 and p.borrow_vectors == 0


@pytest.mark.parametrize("n,d,kw,msg", [
    (0, 8, {}, "n must"),
    (10, 0, {}, "d must"),
    (10, 8, {"nlist": 11}, "nlist"),
    (10, 8, {"nlist": 0}, "nlist"),
    (10, 8, {"bq": 0}, "bq"),
    (10, 8, {"bq": 9}, "bq"),
    (10, 8, {"vectors_on_host": 2}, "vectors_on_host"),
    (10, 8, {"vectors_on_host": -2}, "vectors_on_host"),
    (10, 8, {"borrow_vectors": 2}, "borrow_vectors"),
    (10, 8, {"kmeans_init": 2}, "kmeans_init"),
    (10, 8, {"ivf_flat": 2}, "ivf_flat"),
    (10, 8, {"borrow_vectors": 1, "vectors_on_host": 0}, "borrow_vectors needs the vectors on the host"),
])
def test_build_rejects_bad_arguments(n, d, kw, msg):
    L = rbq.lib()
    x = np.zeros((max(n, 1), max(d, 1)), np.float32)
    p = _params(**kw)
    h = C.c_void_p()
    st = L.rbq_build_index(x.ctypes.data, n, d, C.byref(p), C.byref(h))
    assert st == rbq.RBQ_EINVAL
    assert msg in L.rbq_last_error().decode()
    assert not h.value


def test_build_rejects_nonzero_reserved():
    L = rbq.lib()
    x = np.zeros((10, 8), np.float32)
    p = _params()
    p.reserved[2] = 1
    h = C.c_void_p()
    assert L.rbq_build_index(x.ctypes.data, 10, 8, C.byref(p), C.byref(h)) == rbq.RBQ_EINVAL


def test_null_arguments():
    L = rbq.lib()
    x = np.zeros((10, 8), np.float32)
    p = _params()
    h = C.c_void_p()
    assert L.rbq_build_index(None, 10, 8, C.byref(p), C.byref(h)) == rbq.RBQ_EINVAL
    assert L.rbq_build_index(x.ctypes.data, 10, 8, None, C.byref(h)) == rbq.RBQ_EINVAL
    assert L.rbq_build_index(x.ctypes.data, 10, 8, C.byref(p), None) == rbq.RBQ_EINVAL
    ids = np.zeros(10, np.int64)
    dist = np.zeros(10, np.float32)
    assert L.rbq_search(None, x.ctypes.data, 1, 1, 1, 1, ids.ctypes.data, dist.ctypes.data, None) == rbq.RBQ_EINVAL
    assert "index is NULL" in L.rbq_last_error().decode()
    assert L.rbq_free_index(None) == rbq.RBQ_EINVAL
    assert L.rbq_export(None, 1, x.ctypes.data, 4) == rbq.RBQ_EINVAL
    assert L.rbq_set_timing(None, 1) == rbq.RBQ_EINVAL
    t = rbq.Timings()
    assert L.rbq_get_timings(None, C.byref(t)) == rbq.RBQ_EINVAL
    assert L.rbq_save(None, b"/tmp/x") == rbq.RBQ_EINVAL
    assert L.rbq_load(None, C.byref(h)) == rbq.RBQ_EINVAL
    info = rbq.IndexInfo()
    assert L.rbq_get_info(None, C.byref(info)) == rbq.RBQ_EINVAL


def test_struct_sizes_match_header_layout():
    # natural C layout of the public structs (x86-64 / LP64)
    assert C.sizeof(rbq.BuildParams) == 4 + 4 + 8 + 4 + 4 + 8 + 3 * 8 + 4 + 4 + 4 + 4 + 4 + 3 * 4
    assert C.sizeof(rbq.DebugIO) == 14 * 8 + 8 + 8
    assert C.sizeof(rbq.Timings) == 8 + 7 * 4 + 4 + 5 * 8 + 4 + 4 + 2 * 8 + 8 + 4 + 4 + 2 * 8 + 8
    assert C.sizeof(rbq.IndexInfo) == 8 + 4 * 4 + 3 * 8 + 4 + 4
    assert C.sizeof(rbq.ServerParams) == 6 * 4 + 8 + 8 * 4
    assert C.sizeof(rbq.ServerStats) == 8 * 8
    assert C.sizeof(rbq.ReplayIO) == 8 * 8 + 8 + 4 + 4
    assert C.sizeof(rbq.TuneResult) == 4 * 4 + 2 * 4 + 4 + 4 + 4 + 4 + 4 + 4


def test_tuning_null_arguments():
    L = rbq.lib()
    q = np.zeros((2, 8), np.float32)
    r = rbq.TuneResult()
    assert L.rbq_autotune(None, q.ctypes.data, 2, 1, 1, 1, C.byref(r)) == rbq.RBQ_EINVAL
    assert L.rbq_tune_save(None, b"/tmp/x") == rbq.RBQ_EINVAL
    n = C.c_int32()
    assert L.rbq_tune_load(None, b"/tmp/x", C.byref(n)) == rbq.RBQ_EINVAL
    assert L.rbq_tune_clear(None) == rbq.RBQ_EINVAL


def test_server_params_defaults():
    p = rbq.ServerParams()
    assert rbq.lib().rbq_server_params_init(C.byref(p)) == rbq.RBQ_OK
    assert (p.lanes, p.max_batch, p.queue_cap, p.max_nprobe, p.max_k, p.max_rerank) == (
        2, 1024, 65536, 0, 100, 1000)
    assert p.mem_budget == 1 << 30 and list(p.reserved) == [0] * 8
    assert rbq.lib().rbq_server_params_init(None) == rbq.RBQ_EINVAL


def test_serving_and_mixed_null_arguments():
    L = rbq.lib()
    p = rbq.ServerParams()
    L.rbq_server_params_init(C.byref(p))
    h = C.c_void_p()
    assert L.rbq_server_create(None, C.byref(p), C.byref(h)) == rbq.RBQ_EINVAL
    assert not h.value
    q = np.zeros(8, np.float32)
    t = C.c_uint64()
    assert L.rbq_submit(None, q.ctypes.data, 1, 1, 1, C.byref(t)) == rbq.RBQ_EINVAL
    ids = np.zeros(4, np.int64)
    dist = np.zeros(4, np.float32)
    done = C.c_int32()
    assert L.rbq_poll(None, 0, ids.ctypes.data, dist.ctypes.data, C.byref(done), None) == rbq.RBQ_EINVAL
    assert L.rbq_wait(None, 0, ids.ctypes.data, dist.ctypes.data, 0, None) == rbq.RBQ_EINVAL
    st = rbq.ServerStats()
    assert L.rbq_server_get_stats(None, C.byref(st)) == rbq.RBQ_EINVAL
    assert L.rbq_server_destroy(None) == rbq.RBQ_EINVAL
    io = rbq.ReplayIO()
    assert L.rbq_server_replay(None, C.byref(io)) == rbq.RBQ_EINVAL
    assert L.rbq_replay_plain(None, C.byref(io)) == rbq.RBQ_EINVAL
    a = np.ones(2, np.int32)
    assert L.rbq_search_mixed(None, q.ctypes.data, 1, a.ctypes.data, a.ctypes.data, a.ctypes.data,
                              1, ids.ctypes.data, dist.ctypes.data, None) == rbq.RBQ_EINVAL
    assert "index is NULL" in L.rbq_last_error().decode()
