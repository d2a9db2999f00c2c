"""GPU tests of mixed batches and the continuous-batching server.

Each query's result must not depend on the rest of its batch: probing,
estimates, the exact top-rerank_n selection and the re-rank are per query, so a
query in a mixed batch or in the server's batches returns bit-for-bit what
rbq_search returns for it alone with its own (nprobe, k, rerank_n). The alone
results themselves are pinned to the oracle by the parity tests; a few are
re-checked against the oracle here under the P7 rule.
"""
import ctypes as C
import math
import sys
import threading

import numpy as np
import pytest

import oracle as O
from paper_2605_16007_amd import RbqError, Server
from paper_2605_16007_amd import rbq
from tests._parity import est_scale, lib_index, make_case, set_diff_ok

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    _say("[serving] mixture n=30000 d=128 nlist=64 nq=240")
    X, Q, idx = make_case(30_000, 128, 64, 240, seed=31)
    lib = lib_index(X, idx)
    rng = np.random.default_rng(5)
    nq = len(Q)
    nprobe = rng.choice([1, 2, 3, 8, 16, 33, 64], nq).astype(np.int32)
    k = rng.choice([1, 10, 37, 100], nq).astype(np.int32)
    R = np.maximum(k, rng.choice([1, 10, 100, 250, 1000], nq)).astype(np.int32)
    alone_ids, alone_d = [], []
    for i in range(nq):
        a, b = lib.search(Q[i:i + 1], int(nprobe[i]), int(k[i]), int(R[i]))
        alone_ids.append(a[0])
        alone_d.append(b[0])
    yield dict(X=X, Q=Q, idx=idx, lib=lib, nprobe=nprobe, k=k, R=R, alone_ids=alone_ids,
               alone_d=alone_d)
    lib.close()


def _check_rows(c, ids, dists, rows=None):
    rows = range(len(c["Q"])) if rows is None else rows
    for t, i in enumerate(rows):
        kr = int(c["k"][i])
        np.testing.assert_array_equal(ids[t][:kr], c["alone_ids"][i], err_msg=f"query {i}")
        np.testing.assert_array_equal(dists[t][:kr], c["alone_d"][i], err_msg=f"query {i}")
        assert np.all(ids[t][kr:] == -1) and np.all(np.isinf(dists[t][kr:]))


@pytest.mark.parametrize("scan", [0, 1, 2])
def test_mixed_batch_equals_alone(case, scan):
    _say(f"[serving] mixed batch, scan mode {scan}")
    lib = case["lib"]
    lib.set_option("scan", scan)
    try:
        ids, dists = lib.search_mixed(case["Q"], case["nprobe"], case["k"], case["R"])
    finally:
        lib.set_option("scan", 0)
    _check_rows(case, ids, dists)


def test_mixed_batch_on_device(case):
    import torch
    _say("[serving] mixed batch with device tensors on a side stream")
    lib = case["lib"]
    q = torch.from_numpy(case["Q"]).cuda()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ids, dists = lib.search_mixed(q, case["nprobe"], case["k"], case["R"])
    s.synchronize()
    _check_rows(case, ids.cpu().numpy(), dists.cpu().numpy())


def test_alone_results_match_oracle(case):
    """A few mixed-parameter queries against the oracle under the P7 rule: the
    final ids agree except for exact-distance ties within 1e-5 relative, or
    ids whose oracle estimate ties the rerank_n-th candidate's (P6 near-tie);
    every returned distance is the exact one within FP32 rounding."""
    X, Q, idx = case["X"], case["Q"], case["idx"]
    d = X.shape[1]
    for i in range(0, len(Q), 40):
        npb, kr, R = int(case["nprobe"][i]), int(case["k"][i]), int(case["R"][i])
        _say(f"[serving] oracle check query {i} nprobe={npb} k={kr} R={R}")
        ref_ids, ref_d, st = O.search(idx, X, Q[i:i + 1], npb, kr, R, stages=True)
        val, tol = {}, {}
        for p, pl in enumerate(st["per_list"][0]):
            S = est_scale(st["rnorm2"][0][p], st["vl"][0][p], st["delta"][0][p],
                          st["sumqu"][0][p], pl["ip"], pl["pop"], idx.n_x[pl["ids"]],
                          idx.alpha[pl["ids"]], d)
            for v, e, sc in zip(pl["ids"].tolist(), pl["est"].tolist(), S.tolist()):
                val[v], tol[v] = e, 2e-5 * sc
        exact = lambda x: float(np.sum((X[x].astype(np.float64) - Q[i].astype(np.float64)) ** 2))
        ok = ref_ids[0][ref_ids[0] >= 0]
        boundary = ref_d[0][len(ok) - 1] if len(ok) else math.inf
        cand_boundary = st["cand_est"][0][-1]

        def tol_of(x):
            if x in val and abs(val[x] - cand_boundary) <= tol[x]:
                return math.inf
            return 1e-5 * max(exact(x), boundary) + 1e-6
        g, gd = case["alone_ids"][i], case["alone_d"][i]
        bad = set_diff_ok(g, ref_ids[0], exact, boundary, tol_of)
        assert not bad, (i, bad[:5])
        for v, dist in zip(g.tolist(), gd.tolist()):
            if v >= 0:
                assert abs(dist - exact(v)) <= 4 * d * 2.0 ** -24 * exact(v) + 1e-30


def test_server_mix_equals_alone(case):
    _say("[serving] server, 2 lanes, max_batch 48, burst replay")
    Q = case["Q"]
    arr = np.zeros(len(Q))
    arr[len(Q) // 2:] = 0.002  # two bursts: the second arrives while the first runs
    with Server(case["lib"], lanes=2, max_batch=48, max_nprobe=64, max_k=100,
                max_rerank=1000, mem_budget=256 << 20) as srv:
        ids, dists, lat = srv.replay(Q, case["nprobe"], case["k"], case["R"], arr)
        st = srv.stats()
    _say(f"[serving] stats {st}")
    _check_rows(case, ids, dists)
    assert np.all(np.isfinite(lat)) and np.all(lat >= 0)
    assert st["completed"] == len(Q) and st["batches"] >= len(Q) // 48
    assert st["max_batch_seen"] > 1  # requests were batched


def test_server_memory_admission(case):
    """A budget that holds only a few requests cuts batches short; results do
    not change."""
    _say("[serving] server with a small memory budget")
    Q = case["Q"]
    with Server(case["lib"], lanes=1, max_batch=1024, max_nprobe=64, max_k=100,
                max_rerank=1000, mem_budget=2 << 20) as srv:
        ids, dists, _ = srv.replay(Q, case["nprobe"], case["k"], case["R"], np.zeros(len(Q)))
        st = srv.stats()
    _say(f"[serving] stats {st}")
    _check_rows(case, ids, dists)
    assert st["budget_cuts"] > 0 and st["max_batch_seen"] < len(Q)


@pytest.mark.parametrize("budget_mb", [3, 5, 8, 12, 20])
def test_server_budget_limits_the_pool(case, budget_mb):
    """Budgets at which the candidate pool is the limiting term, with rerank_n
    (1000) above the average list length (469) over the first chunk factor:
    the schedule at the pool budget a lane picks may hold list-major chunks
    that the smallest pool's schedule has not; the lane sizes the whole
    workspace at the budget it uses, so every batch runs and results equal the
    alone ones."""
    Q = case["Q"][:120]
    rows = list(range(120))
    npb = np.full(120, 64, np.int32)
    k = np.full(120, 100, np.int32)
    R = np.full(120, 1000, np.int32)
    alone = [case["lib"].search(Q[i:i + 1], 64, 100, 1000) for i in range(0, 120, 17)]
    with Server(case["lib"], lanes=1, max_batch=1024, max_nprobe=64, max_k=100,
                max_rerank=1000, mem_budget=budget_mb << 20) as srv:
        ids, dists, _ = srv.replay(Q, npb, k, R, np.zeros(120))
        st = srv.stats()
    _say(f"[serving] budget {budget_mb} MB: {st}")
    assert st["completed"] == 120
    for t, i in enumerate(range(0, 120, 17)):
        np.testing.assert_array_equal(ids[i], alone[t][0][0])
        np.testing.assert_array_equal(dists[i], alone[t][1][0])


def test_server_concurrent_submitters(case):
    _say("[serving] 4 submitting threads, poll and wait")
    Q = case["Q"]
    out = {}
    errors = []
    with Server(case["lib"], lanes=2, max_batch=32, max_nprobe=64) as srv:
        def worker(rows):
            try:
                tickets = []
                for i in rows:
                    t = srv.submit(Q[i], case["nprobe"][i], case["k"][i], case["R"][i])
                    assert t is not None
                    tickets.append((i, t))
                for n, (i, t) in enumerate(tickets):
                    if n % 2:
                        r = srv.wait(t, int(case["k"][i]))
                    else:
                        r = None
                        while r is None:
                            r = srv.poll(t, int(case["k"][i]))
                    out[i] = r
            except Exception as e:  # surfaced below
                errors.append(e)
        th = [threading.Thread(target=worker, args=(range(w, len(Q), 4),)) for w in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    assert not errors, errors
    rows = sorted(out)
    assert rows == list(range(len(Q)))
    kmax = int(case["k"].max())
    ids = np.full((len(Q), kmax), -1, np.int64)
    dd = np.full((len(Q), kmax), np.inf, np.float32)
    for i in rows:
        kr = int(case["k"][i])
        ids[i, :kr], dd[i, :kr] = out[i][0], out[i][1]
        assert out[i][2] >= 0
    _check_rows(case, ids, dd)


def test_server_ticket_and_argument_errors(case):
    _say("[serving] tickets, queue limit, argument errors")
    Q, lib = case["Q"], case["lib"]
    with pytest.raises(RbqError) as e:
        Server(lib, max_nprobe=65)  # above nlist
    assert e.value.status == rbq.RBQ_EINVAL
    with pytest.raises(RbqError) as e:
        Server(lib, max_nprobe=64, mem_budget=1000)
    assert e.value.status == rbq.RBQ_EINVAL and "mem_budget" in str(e.value)
    with Server(lib, lanes=1, queue_cap=3, max_nprobe=64) as srv:
        ts = [srv.submit(Q[i], 4, 10, 50) for i in range(3)]
        assert all(t is not None for t in ts)
        while srv.stats()["completed"] < 3:  # finished but not collected: slots stay held
            pass
        assert srv.submit(Q[3], 4, 10, 50) is None  # RBQ_EAGAIN
        assert srv.stats()["rejected"] == 1
        r0 = srv.wait(ts[0], 10)
        a, b = lib.search(Q[0:1], 4, 10, 50)
        np.testing.assert_array_equal(r0[0], a[0])
        np.testing.assert_array_equal(r0[1], b[0])
        with pytest.raises(RbqError):  # already collected
            srv.poll(ts[0], 10)
        with pytest.raises(RbqError):
            srv.poll(ts[1] ^ (1 << 40), 10)  # wrong generation
        with pytest.raises(RbqError):
            srv.submit(Q[0], 65, 10, 50)  # nprobe above max_nprobe
        with pytest.raises(RbqError):
            srv.submit(Q[0], 4, 60, 50)  # k above rerank_n
        import torch
        qd = torch.from_numpy(Q[0].copy()).cuda()
        t = C.c_uint64()
        st = rbq.lib().rbq_submit(srv._h, qd.data_ptr(), 4, 10, 50, C.byref(t))
        assert st == rbq.RBQ_EINVAL and "host memory" in rbq.lib().rbq_last_error().decode()
        assert srv.submit(Q[3], 4, 10, 50) is not None  # a slot was freed


def test_server_destroy_drains(case):
    _say("[serving] destroy with queued requests")
    Q = case["Q"]
    srv = Server(case["lib"], lanes=2, max_batch=16, max_nprobe=64)
    for i in range(100):
        assert srv.submit(Q[i], case["nprobe"][i], case["k"][i], case["R"][i]) is not None
    srv.close()  # finishes the queued work, then frees


def test_replay_plain_equals_server(case):
    _say("[serving] plain per-query replay")
    Q = case["Q"][:60]
    arr = np.linspace(0, 0.01, len(Q))
    ids, dists, lat = case["lib"].replay_plain(Q, case["nprobe"][:60], case["k"][:60],
                                               case["R"][:60], arr)
    _check_rows(case, ids, dists, rows=range(60))
    assert np.all(np.isfinite(lat)) and np.all(lat >= 0)
