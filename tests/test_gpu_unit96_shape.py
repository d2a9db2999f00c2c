"""Parity in the shape of the 400M x 96 unit-vector workload at a size the
oracle handles: D = 96, nlist = 8192 (probe selection for nlist > 4096),
batches of 2560 queries, raw vectors in pinned host memory borrowed from the
caller, re-rank on host cores in overlapped sub-batches (Sec. 3.3.4), and
list-major scan chunks.

The index is made from oracle parts: 8192 seeded database rows as centroids,
a Haar P and the oracle's FP64 assignment.
Checked:
  * probes of all 2560 queries against the oracle (near-ties of the FP32 probe
    score may swap lists);
  * the un-injected batch: the automatic schedule and the list-major scan for
    every chunk return identical results; the borrowed-host index and an index
    with the vectors in HBM return the same candidates, and final results
    that differ only at exact-distance near-ties; returned distances are the
    FP64 distances rounded once;
  * with the oracle's probes, qu and scalars injected into the whole batch:
    candidate sets (P6) and final ids (P7) of sampled queries against the
    oracle's search.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import est_scale, set_diff_ok

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N, D, NLIST, NQ = 200_000, 96, 8192, 2560
NPROBE, K, R = 64, 10, 100
SAMPLED = (0, 1, 777, 1500, 2047, 2048, 2559)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def case():
    import torch
    from synth import database, get, queries
    from paper_2605_16007_amd import Index
    w = get("unit96_400m", n=N, nlist=NLIST, nq=NQ, centres=NLIST // 2)
    _say(f"[unit96] n={N} d={D} nlist={NLIST} batch={NQ} nprobe={NPROBE} R={R}")
    X = database(w)
    Q = queries(w)
    rng = np.random.default_rng(96)
    C = np.asarray(X[np.sort(rng.choice(N, NLIST, replace=False))], np.float32)
    P = O.random_orthogonal(D, rng).astype(np.float32)
    a, _ = O.assign(X, C)
    oidx = O.build(X, NLIST, centroids=C, P=P, assignment=a)
    _say("[unit96] oracle index ready; building the library indexes")
    xp = torch.empty((N, D), dtype=torch.float32, pin_memory=True)
    xp.numpy()[:] = X
    host = Index.build(xp, NLIST, centroids=C, rotation=P, assignment=a.astype(np.int32),
                       vectors_on_host=True, borrow_vectors=True)
    dev = Index.build(X, NLIST, centroids=C, rotation=P, assignment=a.astype(np.int32),
                      vectors_on_host=False)
    yield dict(X=X, Q=Q, C=C, P=P, oidx=oidx, host=host, dev=dev, xp=xp)
    host.close()
    dev.close()


def test_borrowed_index_info(case):
    inf = case["host"].info()
    assert inf["vectors_on_host"] == 1 and inf["vectors_borrowed"] == 1
    assert case["dev"].info()["vectors_on_host"] == 0 and case["dev"].info()["vectors_borrowed"] == 0
    np.testing.assert_array_equal(case["host"].export("codes"), case["oidx"].codes)


def test_probes_nlist_8192(case):
    Q, C = case["Q"], case["C"]
    got = case["host"].search_debug(Q, NPROBE, K, R, want={"probes"})["probes"]
    cn = np.sum(C.astype(np.float64) ** 2, axis=1)
    mism = 0
    for i in range(NQ):
        pr, pd = O.probe(Q[i], C, NPROBE)
        if np.array_equal(got[i], pr):
            continue
        mism += 1
        dist = lambda j: float(np.sum((C[j].astype(np.float64) - Q[i]) ** 2))
        tol = lambda j: 4 * D * 2.0 ** -24 * (cn[j] + 2 * math.sqrt(cn[j]) * float(np.linalg.norm(Q[i]))) + 1e-6
        bad = set_diff_ok(got[i], pr, dist, pd[-1], tol)
        assert not bad, (i, bad[:5])
    _say(f"[unit96] probes: {NQ - mism} of {NQ} queries identical, the rest differ at near-ties")


def _exact(X, q, i):
    return float(np.sum((X[i].astype(np.float64) - q.astype(np.float64)) ** 2))


def test_batch_schedules_and_placements_agree(case):
    host, dev, X, Q = case["host"], case["dev"], case["X"], case["Q"]
    outs = {}
    for scan in (0, 2):
        host.set_option("scan", scan)
        host.set_timing(True)
        try:
            outs[scan] = host.search(Q, NPROBE, K, R)  # four overlapped sub-batches
            t = host.timings()
        finally:
            host.set_timing(False)
            host.set_option("scan", 0)
        _say(f"[unit96] scan {scan}: {t['group_launches']} list-major, {t['popc_launches']} query-major launches")
        if scan == 2:
            assert t["group_launches"] > 0 and t["popc_launches"] == 0, t
    np.testing.assert_array_equal(outs[0][0], outs[2][0])
    np.testing.assert_array_equal(outs[0][1], outs[2][1])
    ids, dd = outs[0]
    want = {"cand_ids", "cand_est"}
    a = host.search_debug(Q, NPROBE, K, R, want=want)
    b = dev.search_debug(Q, NPROBE, K, R, want=want)
    for key in want:
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)
    d_ids, d_d = dev.search(Q, NPROBE, K, R)
    for qi in range(NQ):
        assert np.all(ids[qi] >= 0) and np.all(np.diff(dd[qi]) >= 0)
        for x, y in zip(ids[qi], d_ids[qi]):
            if x != y:
                ex, ey = _exact(X, Q[qi], x), _exact(X, Q[qi], y)
                assert abs(ex - ey) <= 8 * D * 2.0 ** -24 * max(ex, ey), (qi, x, y, ex, ey)
    for qi in range(0, NQ, 37):
        for i, dist in zip(ids[qi].tolist(), dd[qi].tolist()):
            e = _exact(X, Q[qi], i)
            assert abs(dist - e) <= 2.0 ** -24 * e


def test_injected_batch_p6_p7(case):
    host, X, Q, C, P, oidx = case["host"], case["X"], case["Q"], case["C"], case["P"], case["oidx"]
    _say("[unit96] oracle probes and quantised residuals of the whole batch")
    Cr = C.astype(np.float64) @ P.astype(np.float64)
    probes = np.empty((NQ, NPROBE), np.int32)
    qu = np.empty((NQ, NPROBE, D), np.uint8)
    sc = np.empty((NQ, NPROBE, 3), np.float32)
    for i in range(NQ):
        pr, _ = O.probe(Q[i], C, NPROBE)
        probes[i] = pr
        qrot = O.rotate(Q[i], P)
        for p, j in enumerate(pr):
            r = qrot - Cr[j]
            u, vl, delta, _ = O.quantize(r, oidx.bq)
            qu[i, p] = u
            sc[i, p] = (float(r @ r), vl, delta)
    host.set_option("scan", 2)
    try:
        out = host.search_debug(Q, NPROBE, K, R, inject_probes=probes, inject_qu=qu, inject_scalars=sc,
                                want={"cand_ids", "cand_est", "ids", "sqdist"})
    finally:
        host.set_option("scan", 0)
    rows = list(SAMPLED)
    ref_ids, ref_d, st = O.search(oidx, X, Q[rows], NPROBE, K, R, stages=True)
    for t, qi in enumerate(rows):
        val, tol = {}, {}
        for p, pl in enumerate(st["per_list"][t]):
            S = est_scale(st["rnorm2"][t][p], st["vl"][t][p], st["delta"][t][p], st["sumqu"][t][p],
                          pl["ip"], pl["pop"], oidx.n_x[pl["ids"]], oidx.alpha[pl["ids"]], D)
            for i, e, s in zip(pl["ids"].tolist(), pl["est"].tolist(), S.tolist()):
                val[i], tol[i] = e, s
        ref = st["cand_ids"][t]
        rv = ref[ref >= 0]
        boundary = val[int(rv[-1])]
        bad = set_diff_ok(out["cand_ids"][qi], ref, lambda x: val[x], boundary, lambda x: 2e-5 * tol[x])
        assert not bad, ("P6", qi, bad[:5])
        for x, e in zip(out["cand_ids"][qi].tolist(), out["cand_est"][qi].tolist()):
            if x >= 0:
                assert abs(e - val[x]) <= 1e-5 * tol[x], ("P5", qi, x)
        exact = lambda x: _exact(X, Q[qi], x)
        fb = ref_d[t][-1]

        def tol7(x):
            if x in val and abs(val[x] - boundary) <= 2e-5 * tol[x]:
                return math.inf  # a P6 near-tie at the candidate boundary
            return 1e-5 * max(exact(x), fb) + 1e-6
        bad = set_diff_ok(out["ids"][qi], ref_ids[t], exact, fb, tol7)
        assert not bad, ("P7", qi, bad[:5])
