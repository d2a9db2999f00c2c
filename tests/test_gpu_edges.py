"""GPU edge cases and invariants of the search path (oracle inputs only)."""
import os
import sys
import tempfile

import numpy as np
import pytest

import oracle as O
from tests._parity import lib_index, make_case

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _exact(X, q, i):
    return float(np.sum((X[i].astype(np.float64) - q.astype(np.float64)) ** 2))


def test_reduces_to_exact_knn():
    """Every list probed and every vector re-ranked: exact kNN (Sec. 2.1.1)."""
    _say("[edge] exact kNN reduction n=1500 d=32 nlist=16")
    X, Q, idx = make_case(1500, 32, 16, 21, seed=5)
    lib = lib_index(X, idx)
    ids, dd = lib.search(Q, 16, 10, 1500)
    gt, gd = O.brute_force_knn(X, Q, 10)
    for qi in range(len(Q)):
        if not np.array_equal(ids[qi], gt[qi]):
            # only exact-distance near-ties may reorder
            for a, b in zip(ids[qi], gt[qi]):
                if a != b:
                    assert abs(_exact(X, Q[qi], a) - _exact(X, Q[qi], b)) <= 1e-5 * _exact(X, Q[qi], b)
        np.testing.assert_allclose(dd[qi], gd[qi], rtol=4 * 32 * 2.0 ** -24)


def test_empty_lists_zero_residual_and_padding():
    """Probed lists that are empty, vectors equal to their centroid (n_x = 0),
    fewer candidates than rerank_n (padding with -1 / +inf)."""
    _say("[edge] empty lists / n_x = 0 / padding")
    rng = np.random.default_rng(7)
    d, nlist = 24, 10
    C = rng.normal(size=(nlist, d)).astype(np.float32)
    C[7:] += 1000.0                      # lists 7..9 stay empty
    lab = rng.integers(0, 7, 300)
    X = (C[lab] + 0.1 * rng.normal(size=(300, d))).astype(np.float32)
    X[:5] = C[lab[:5]]                   # exact centroid copies: n_x = 0
    P = O.random_orthogonal(d, rng).astype(np.float32)
    a, _ = O.assign(X, C)
    idx = O.build(X, nlist, centroids=C, P=P, assignment=a)
    assert all(len(idx.lists[j]) == 0 for j in (7, 8, 9))
    lib = lib_index(X, idx)
    f = lib.export("factors")
    assert np.all(f[:5, 0] == 0) and np.all(f[:5, 1] == 1)
    np.testing.assert_array_equal(lib.export("codes")[:5], idx.codes[:5])
    Q = X[:6] + 0.01
    probes = np.array([[7, 8, 9, lab[i]] for i in range(6)], np.int32)
    ref = O.search(idx, X, Q, 4, 8, 700, probes=probes)
    out = lib.search_debug(Q, 4, 8, 700, inject_probes=probes, want={"cand_ids", "ids", "sqdist"})
    for qi in range(6):
        m = len(idx.lists[lab[qi]])
        assert np.all(out["cand_ids"][qi][m:] == -1)
        assert set(out["cand_ids"][qi][:m].tolist()) == set(idx.lists[lab[qi]].tolist())
        np.testing.assert_array_equal(out["ids"][qi], ref[0][qi])
    # k larger than the candidates: padding in the final results too
    out = lib.search_debug(Q[:1], 1, 50, 60, inject_probes=np.array([[8]], np.int32),
                           want={"ids", "sqdist"})
    assert np.all(out["ids"] == -1) and np.all(np.isinf(out["sqdist"]))


def test_probe_chunking_is_invisible():
    """Scanning the probe ranks in chunks (running top-R merged after each)
    returns exactly the same candidates and results."""
    _say("[edge] probe chunking")
    X, Q, idx = make_case(20000, 64, 40, 19, seed=8)
    lib = lib_index(X, idx)
    want = {"cand_ids", "cand_est", "ids", "sqdist"}
    base = lib.search_debug(Q, 12, 10, 90, want=want)
    for ch in (1, 5):
        out = lib.search_debug(Q, 12, 10, 90, want=want, probe_chunk=ch)
        for key in want:
            np.testing.assert_array_equal(out[key], base[key], err_msg=f"{key} chunk {ch}")


def test_single_probe_and_k_equals_R():
    _say("[edge] nprobe = 1, k = rerank_n")
    X, Q, idx = make_case(8000, 48, 20, 13, seed=9)
    lib = lib_index(X, idx)
    ids, dd = lib.search(Q, 1, 30, 30)
    ref_ids, ref_d = O.search(idx, X, Q, 1, 30, 30)
    for qi in range(len(Q)):
        assert set(ids[qi].tolist()) == set(ref_ids[qi].tolist())


def test_device_tensors_match_host_path_and_nq0():
    import torch
    _say("[edge] torch device tensors vs host arrays")
    X, Q, idx = make_case(12000, 128, 32, 33, seed=10)
    lib = lib_index(X, idx)
    ids_h, d_h = lib.search(Q, 6, 10, 100)
    dev = torch.device("cuda:0")
    ids_d, d_d = lib.search(torch.from_numpy(Q).to(dev), 6, 10, 100)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ids_d.cpu().numpy(), ids_h)
    np.testing.assert_array_equal(d_d.cpu().numpy(), d_h)
    # a non-default stream
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        ids_s, d_s = lib.search(torch.from_numpy(Q).to(dev), 6, 10, 100)
    st.synchronize()
    np.testing.assert_array_equal(ids_s.cpu().numpy(), ids_h)
    e_ids, e_d = lib.search(Q[:0], 6, 10, 100)
    assert e_ids.shape == (0, 10)


def test_save_load_roundtrip():
    _say("[edge] save / load")
    X, Q, idx = make_case(6000, 40, 16, 9, seed=11)
    lib = lib_index(X, idx)
    from paper_2605_16007_amd import Index
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "idx.rbq")
        lib.save(path)
        lib2 = Index.load(path)
        for what in ("codes", "factors", "assign", "centroids", "rotation", "list_sizes"):
            np.testing.assert_array_equal(lib2.export(what), lib.export(what))
        a = lib.search(Q, 4, 5, 50)
        b = lib2.search(Q, 4, 5, 50)
        np.testing.assert_array_equal(a[0], b[0])
        np.testing.assert_array_equal(a[1], b[1])
        with open(path, "r+b") as f:     # corrupt one byte of the last section
            f.seek(-3, 2)
            byte = f.read(1)
            f.seek(-3, 2)
            f.write(bytes([byte[0] ^ 0xFF]))
        from paper_2605_16007_amd import RbqError
        with pytest.raises(RbqError, match="checksum"):
            Index.load(path)


def test_library_kmeans_and_rotation_properties():
    """The library's own build (k-means on the GPU, its own Haar P): P is
    orthogonal, every vector sits in its nearest list (up to FP32 near-ties),
    and search quality is sane."""
    _say("[edge] library-built index")
    from synth import get, database, queries
    from paper_2605_16007_amd import Index
    w = get("mixture128", n=20000, nq=16, nlist=64, centres=64)
    X, Q = database(w), queries(w)
    lib = Index.build(X, 64, seed=3, kmeans_iters=10, kmeans_restarts=2)
    P = lib.export("rotation").astype(np.float64)
    assert np.max(np.abs(P.T @ P - np.eye(128))) < 1e-5
    C = lib.export("centroids").astype(np.float64)
    a = lib.export("assign")
    D = O.sqdist(X, C)
    best = D.min(axis=1)
    mine = D[np.arange(len(X)), a]
    tol = 8 * 128 * 2.0 ** -24 * (np.sum(X.astype(np.float64) ** 2, 1) + np.max(np.sum(C * C, 1)))
    assert np.all(mine - best <= tol)
    assert np.all(lib.export("list_sizes") == np.bincount(a, minlength=64))
    ids, _ = lib.search(Q, 16, 10, 200)
    gt, _ = O.brute_force_knn(X, Q, 10)
    rec = np.mean([len(set(x) & set(y)) / 10 for x, y in zip(ids.tolist(), gt.tolist())])
    assert rec >= 0.9, rec


def test_search_rejects_bad_arguments_on_gpu_index():
    from paper_2605_16007_amd import RbqError
    X, Q, idx = make_case(3000, 16, 8, 4, seed=12)
    lib = lib_index(X, idx)
    for args in ((0, 5, 10), (9, 5, 10), (4, 11, 10), (4, 0, 10), (4, 5, 3841)):
        with pytest.raises(RbqError, match="status -1"):
            lib.search(Q, *args)


def test_large_k_rerank():
    """k = rerank_n at the largest allowed size (the re-rank sorts all
    candidates in place) and a large k below it (radix select path)."""
    _say("[edge] large k")
    X, Q, idx = make_case(6000, 32, 4, 5, seed=13)
    lib = lib_index(X, idx)
    for k, R in ((3840, 3840), (2900, 3000)):
        ids, dd = lib.search(Q, 4, k, R)
        ref_ids, ref_d = O.search(idx, X, Q, 4, k, R)
        for qi in range(len(Q)):
            g = ids[qi]
            assert np.all(np.diff(dd[qi][g >= 0]) >= 0)
            common = len(set(g.tolist()) & set(ref_ids[qi].tolist()))
            assert common >= k - 5, (k, qi, common)


def test_many_searches_in_flight_reuse_workspaces():
    """Searches that only enqueue (raw vectors in HBM, device outputs) can be
    issued faster than the GPU completes them; past a few held workspaces a
    search waits for the oldest instead of allocating another. Sixteen
    back-to-back searches on one stream equal the same search run alone."""
    import torch
    _say("[edge] 16 searches in flight n=20000 d=64 nlist=64")
    X, Q, idx = make_case(20_000, 64, 64, 400, seed=13)
    lib = lib_index(X, idx)
    try:
        q = torch.from_numpy(Q).cuda()
        ref_ids, ref_d = lib.search(q, 16, 10, 200)
        torch.cuda.synchronize()
        outs = [(torch.empty((len(Q), 10), dtype=torch.int64, device="cuda"),
                 torch.empty((len(Q), 10), dtype=torch.float32, device="cuda")) for _ in range(16)]
        st = torch.cuda.Stream()
        for oi, od in outs:
            lib.search(q, 16, 10, 200, ids=oi, dists=od, stream=st.cuda_stream)
        torch.cuda.synchronize()
        for oi, od in outs:
            assert torch.equal(oi, ref_ids) and torch.equal(od, ref_d)
    finally:
        lib.close()


def test_overflow_redo_is_counted_and_exact():
    """A tiny list-major pool makes queries overflow: they are searched again
    from scratch, the instrumented pass counts them, and the results equal
    those of an ample pool."""
    _say("[edge] pool overflow redo n=20000 d=64 nlist=32")
    X, Q, idx = make_case(20_000, 64, 32, 300, seed=17)
    lib = lib_index(X, idx)
    try:
        lib.set_option("scan", 2)
        ref = lib.search(Q, 8, 10, 100)
        lib.set_timing(True)
        lib.search(Q, 8, 10, 100)
        assert lib.timings()["redo_queries"] == 0
        lib.set_option("pool_cap", 64)
        lib.set_timing(True)
        got = lib.search(Q, 8, 10, 100)
        t = lib.timings()
        lib.set_timing(False)
        assert t["redo_queries"] > 0, t
        np.testing.assert_array_equal(got[0], ref[0])
        np.testing.assert_array_equal(got[1], ref[1])
    finally:
        lib.close()
