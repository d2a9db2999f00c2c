"""GPU tests of the host re-rank path (raw vectors in host memory,
Sec. 3.3.4): the same index built with the vectors on the device and on the
host returns the same candidates; the host path re-ranks them in FP64, so its
final results follow the oracle's exact distances (P7) and differ from the
device re-rank (FP32) only at exact-distance near-ties."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_16007_amd import Index, Server
from tests._parity import lib_index, make_case, set_diff_ok

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pair():
    _say("[host rerank] mixture n=20000 d=96 nlist=32 nq=2100")
    X, Q, idx = make_case(20_000, 96, 32, 2100, seed=41, kind="unit_mixture")
    dev = lib_index(X, idx)
    host = Index.build(X, idx.nlist, centroids=idx.centroids, rotation=idx.P,
                       assignment=idx.assign.astype(np.int32), vectors_on_host=True, host_threads=4)
    yield X, Q, idx, dev, host
    host.close()
    dev.close()


def _exact(X, q, i):
    return float(np.sum((X[i].astype(np.float64) - q.astype(np.float64)) ** 2))


def _same_up_to_ties(X, Q, a_ids, b_ids, b_d, d):
    for qi in range(len(Q)):
        if np.array_equal(a_ids[qi], b_ids[qi]):
            continue
        for x, y in zip(a_ids[qi], b_ids[qi]):
            if x != y:
                assert x >= 0 and y >= 0, (qi, x, y)
                ex, ey = _exact(X, Q[qi], x), _exact(X, Q[qi], y)
                assert abs(ex - ey) <= 8 * d * 2.0 ** -24 * max(ex, ey), (qi, x, y, ex, ey)


def test_info_and_candidates_match_device_index(pair):
    X, Q, idx, dev, host = pair
    assert host.info()["vectors_on_host"] == 1
    np.testing.assert_array_equal(host.export("codes"), dev.export("codes"))
    want = {"cand_ids", "cand_est"}
    a = dev.search_debug(Q[:64], 6, 10, 100, want=want)
    b = host.search_debug(Q[:64], 6, 10, 100, want=want)
    for key in want:
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


@pytest.mark.parametrize("nq", [1, 300, 2100])
def test_host_rerank_matches_device_and_exact(pair, nq):
    """nq 300 and 2100 split the batch into 2 and 4 overlapped sub-batches."""
    X, Q, idx, dev, host = pair
    _say(f"[host rerank] nq={nq}")
    a_ids, a_d = dev.search(Q[:nq], 6, 10, 100)
    b_ids, b_d = host.search(Q[:nq], 6, 10, 100)
    d = X.shape[1]
    _same_up_to_ties(X, Q[:nq], a_ids, b_ids, b_d, d)
    for qi in range(0, nq, max(1, nq // 50)):
        for i, dist in zip(b_ids[qi].tolist(), b_d[qi].tolist()):
            assert i >= 0
            e = _exact(X, Q[qi], i)
            assert abs(dist - e) <= 2.0 ** -24 * e  # the FP64 distance rounded once
        assert np.all(np.diff(b_d[qi]) >= 0)


def test_host_rerank_against_oracle(pair):
    X, Q, idx, dev, host = pair
    _say("[host rerank] oracle P7")
    ref_ids, ref_d, st = O.search(idx, X, Q[:20], 6, 10, 100, stages=True)
    ids, dd = host.search(Q[:20], 6, 10, 100)
    for qi in range(20):
        exact = lambda x: _exact(X, Q[qi], x)
        boundary = ref_d[qi][-1]
        cand = set(int(c) for c in st["cand_ids"][qi])
        # ids may differ only at exact ties or at a coarse-candidate near-tie
        def tol_of(x):
            return 1e-5 * max(exact(x), boundary) + (math.inf if x not in cand else 1e-6)
        bad = set_diff_ok(ids[qi], ref_ids[qi], exact, boundary, tol_of)
        assert not bad, (qi, bad[:5])


def test_host_rerank_device_inputs_and_mixed(pair):
    import torch
    X, Q, idx, dev, host = pair
    _say("[host rerank] device tensors, mixed batch, server")
    q = torch.from_numpy(Q[:500]).cuda()
    ids, dd = host.search(q, 6, 10, 100)
    h_ids, h_d = host.search(Q[:500], 6, 10, 100)
    np.testing.assert_array_equal(ids.cpu().numpy(), h_ids)
    np.testing.assert_array_equal(dd.cpu().numpy(), h_d)
    rng = np.random.default_rng(3)
    npb = rng.integers(1, 33, 500).astype(np.int32)
    k = rng.choice([1, 10, 50], 500).astype(np.int32)
    R = np.maximum(k, rng.choice([10, 100, 400], 500)).astype(np.int32)
    m_ids, m_d = host.search_mixed(Q[:500], npb, k, R)
    for i in range(0, 500, 7):
        a, b = host.search(Q[i:i + 1], int(npb[i]), int(k[i]), int(R[i]))
        np.testing.assert_array_equal(m_ids[i, :k[i]], a[0])
        np.testing.assert_array_equal(m_d[i, :k[i]], b[0])
    with Server(host, lanes=2, max_batch=64, max_nprobe=32, max_k=50, max_rerank=400) as srv:
        s_ids, s_d, _ = srv.replay(Q[:500], npb, k, R, np.zeros(500))
    np.testing.assert_array_equal(s_ids, m_ids)
    np.testing.assert_array_equal(s_d, m_d)


def test_borrowed_and_automatic_placement(pair):
    """borrow_vectors keeps the caller's rows (pinned or pageable, no copy) and
    returns the copied host index's results; automatic placement keeps a small
    index's vectors in HBM; device memory cannot be borrowed."""
    import torch
    from paper_2605_16007_amd.rbq import RbqError
    X, Q, idx, dev, host = pair
    xp = torch.empty(X.shape, dtype=torch.float32, pin_memory=True)
    xp.numpy()[:] = X
    kw = dict(centroids=idx.centroids, rotation=idx.P, assignment=idx.assign.astype(np.int32))
    b = Index.build(xp, idx.nlist, vectors_on_host=True, borrow_vectors=True, host_threads=4, **kw)
    xpage = np.array(X, np.float32, copy=True)
    bp = Index.build(xpage, idx.nlist, vectors_on_host=True, borrow_vectors=True, host_threads=4, **kw)
    auto = Index.build(X, idx.nlist, **kw)
    try:
        assert b.info()["vectors_borrowed"] == 1 and b.info()["vectors_on_host"] == 1
        assert bp.info()["vectors_borrowed"] == 1
        assert host.info()["vectors_borrowed"] == 0
        assert auto.info()["vectors_on_host"] == 0
        for nq in (1, 700, 2100):
            x_ids, x_d = host.search(Q[:nq], 6, 10, 100)
            for ix in (b, bp):
                y_ids, y_d = ix.search(Q[:nq], 6, 10, 100)
                np.testing.assert_array_equal(x_ids, y_ids)
                np.testing.assert_array_equal(x_d, y_d)
        a_ids, a_d = auto.search(Q[:300], 6, 10, 100)
        d_ids, d_d = dev.search(Q[:300], 6, 10, 100)
        np.testing.assert_array_equal(a_ids, d_ids)
        np.testing.assert_array_equal(a_d, d_d)
        with pytest.raises(RbqError, match="not device memory"):
            Index.build(torch.from_numpy(X).cuda(), idx.nlist, vectors_on_host=True,
                        borrow_vectors=True, **kw)
    finally:
        b.close()
        bp.close()
        auto.close()


def test_host_copy_gets_huge_pages(pair):
    """The index's own host rows are private anonymous memory advised for
    transparent huge pages: building a host index of 96 MiB of rows raises the
    process's AnonHugePages by at least half of that."""
    import re
    try:
        mode = re.search(r"\[(\w+)\]", open("/sys/kernel/mm/transparent_hugepage/enabled").read()).group(1)
    except (OSError, AttributeError):
        mode = None
    if mode not in ("always", "madvise"):
        pytest.skip("transparent huge pages are off on this host")
    X, Q, idx, dev, host = pair

    def huge_kb():
        return int(re.search(r"AnonHugePages:\s+(\d+)", open("/proc/self/smaps_rollup").read()).group(1))

    reps = 96 * 2**20 // X.nbytes + 1
    big = np.ascontiguousarray(np.tile(X, (reps, 1)))
    _say(f"[host rerank] host copy of {big.nbytes >> 20} MiB")
    before = huge_kb()
    ix = Index.build(big, idx.nlist, centroids=idx.centroids, rotation=idx.P, vectors_on_host=True,
                     host_threads=4)
    try:
        after = huge_kb()
        assert after - before >= 48 * 1024, (before, after)
        ids, _ = ix.search(Q[:8], 6, 10, 100)
        assert (ids >= 0).all()
    finally:
        ix.close()



def test_host_parts_leave_results_unchanged(pair):
    """RBQ_OPT_HOST_PARTS (sub-batches overlapped with the host re-rank) and
    its automatic rule return the same results for every split."""
    from paper_2605_16007_amd.rbq import RbqError
    X, Q, idx, dev, host = pair
    ref_ids, ref_d = host.search(Q[:2100], 6, 10, 100)
    try:
        for parts in (1, 2, 3, 7, 64):
            host.set_option("host_parts", parts)
            ids, dd = host.search(Q[:2100], 6, 10, 100)
            np.testing.assert_array_equal(ids, ref_ids)
            np.testing.assert_array_equal(dd, ref_d)
        with pytest.raises(RbqError):
            host.set_option("host_parts", 65)
    finally:
        host.set_option("host_parts", 0)


def test_concurrent_callers_match_sequential(pair):
    """Several caller threads searching the host index at once (each on its own
    stream; their GPU parts take turns on the index's host-path stream) get
    the results of the same searches run one after another."""
    import threading
    import torch
    X, Q, idx, dev, host = pair
    slices = [Q[i * 500:(i + 1) * 500] for i in range(4)]
    ref = [host.search(qs, 6, 10, 100) for qs in slices]
    got = [None] * len(slices)
    errs = []

    def run(t):
        try:
            torch.cuda.set_device(0)
            st = torch.cuda.Stream()
            q = torch.from_numpy(slices[t]).cuda()
            torch.cuda.synchronize()
            for _ in range(3):
                ids, dd = host.search(q, 6, 10, 100, stream=st.cuda_stream)
            st.synchronize()
            got[t] = (ids.cpu().numpy(), dd.cpu().numpy())
        except Exception as e:  # reported below
            errs.append(e)

    th = [threading.Thread(target=run, args=(t,)) for t in range(len(slices))]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert not errs, errs
    for (a_ids, a_d), (b_ids, b_d) in zip(ref, got):
        np.testing.assert_array_equal(a_ids, b_ids)
        np.testing.assert_array_equal(a_d, b_d)
