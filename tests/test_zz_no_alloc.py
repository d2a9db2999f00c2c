"""rbq_search_noalloc (the entry point for callers that cannot allocate device
memory) through the C ABI: its results equal rbq_search's on two calls in a
row, the second with a smaller batch, so the reused workspace array carries
nothing from one call into the next; a batch whose smallest workspace exceeds
the array and host pointers are refused with a clear error."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_2605_16007_amd import rbq
from tests._parity import lib_index, make_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    _say("[noalloc] mixture n=40000 d=128 nlist=128 nq=600")
    X, Q, idx = make_case(40_000, 128, 128, 600, seed=77)
    lib = lib_index(X, idx)
    yield X, Q, lib
    lib.close()


def _abi(lib, q, nprobe, k, R):
    """Calls rbq_search_noalloc directly with device tensors."""
    import torch
    nq = q.shape[0]
    ids = torch.full((nq, k), -7, dtype=torch.int64, device=q.device)
    dd = torch.full((nq, k), -7.0, dtype=torch.float32, device=q.device)
    st = rbq.lib().rbq_search_noalloc(lib._h, C.c_void_p(q.data_ptr()), nq, nprobe, k, R,
                                      C.c_void_p(ids.data_ptr()), C.c_void_p(dd.data_ptr()),
                                      C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == rbq.RBQ_OK, rbq.lib().rbq_last_error().decode()
    torch.cuda.synchronize()
    return ids.cpu().numpy(), dd.cpu().numpy()


@pytest.mark.parametrize("nprobe,k,R", [(16, 10, 100), (64, 10, 1000), (128, 100, 3840)])
def test_noalloc_equals_search_twice(case, nprobe, k, R):
    import torch
    X, Q, lib = case
    for nq in (600, 97):  # the second call is smaller and reuses the array
        _say(f"[noalloc] nq={nq} nprobe={nprobe} k={k} R={R}")
        q = torch.from_numpy(Q[:nq]).cuda()
        a_ids, a_d = _abi(lib, q, nprobe, k, R)
        b_ids, b_d = lib.search(Q[:nq], nprobe, k, R)
        np.testing.assert_array_equal(a_ids, b_ids)
        np.testing.assert_array_equal(a_d, b_d)


def test_noalloc_refusals(case):
    import torch
    X, Q, lib = case
    q = torch.from_numpy(Q[:8]).cuda()
    ids = torch.empty((8, 10), dtype=torch.int64, device="cuda")
    dd = torch.empty((8, 10), dtype=torch.float32, device="cuda")
    L = rbq.lib()
    # host queries
    st = L.rbq_search_noalloc(lib._h, C.c_void_p(Q[:8].ctypes.data), 8, 16, 10, 100,
                              C.c_void_p(ids.data_ptr()), C.c_void_p(dd.data_ptr()), None)
    assert st == rbq.RBQ_EINVAL and "device pointers" in L.rbq_last_error().decode()
    # a batch far beyond the array: 40000 queries x 128 probes x 3840 candidates
    big = torch.zeros((40_000, 128), dtype=torch.float32, device="cuda")
    bids = torch.empty((40_000, 10), dtype=torch.int64, device="cuda")
    bdd = torch.empty((40_000, 10), dtype=torch.float32, device="cuda")
    st = L.rbq_search_noalloc(lib._h, C.c_void_p(big.data_ptr()), 40_000, 128, 10, 3840,
                              C.c_void_p(bids.data_ptr()), C.c_void_p(bdd.data_ptr()), None)
    assert st == rbq.RBQ_EINVAL
    msg = L.rbq_last_error().decode()
    assert "256 MiB" in msg and "split" in msg, msg
    # still usable afterwards
    a_ids, a_d = _abi(lib, q, 16, 10, 100)
    b_ids, b_d = lib.search(Q[:8], 16, 10, 100)
    np.testing.assert_array_equal(a_ids, b_ids)
    np.testing.assert_array_equal(a_d, b_d)
