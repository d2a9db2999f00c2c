"""Parity at full size, in the launch configuration the benchmark times:
10M x 128 skewed integer vectors, nlist 4096, one batch of 1024 queries,
nprobe 512, rerank_n 3840, k 10, B_q 4 (query-major popcount scan for the
leading small chunks of probe ranks, the list-major fp4 x fp8 matrix-core scan
for the rest).

The oracle cannot build a 10M-vector index in a test's time, so the index is
made from oracle parts: centroids from two Lloyd steps (FP64) started at 4096
seeded database rows, and a Haar P; the library assigns the vectors (its GPU
argmin). Checked here:
  * sampled queries, one by one, against the oracle: probes; with the oracle's
    probes, qu and scalars injected into the full batch, the candidate set (P6)
    and the final top-k (P7); with the same injection for the sampled queries
    alone, every integer inner product (P4, bit-exact) and every estimate (P5)
    of all their 512 probed lists, against the oracle's own FP64 encoding of
    the lists' members;
  * list membership: every member of 16 sampled probed lists per sampled query
    has that list's centroid as its FP64 nearest one (ties within FP32 error
    allowed), and every vector is in exactly one list;
  * for all 1024 queries of the un-injected batch: returned distances are the
    exact ones (FP32-rounded), ascending, ids distinct; the list-major and the
    query-major scans return identical candidates and results.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import est_scale, set_diff_ok

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

NPROBE, K, R = 512, 10, 3840
SAMPLED = (0, 517, 1023)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full():
    from synth import database, get, queries
    from paper_2605_16007_amd import Index
    w = get("sift10m")
    _say(f"[fullsize] {w.name}: n={w.n} d={w.d} nlist={w.nlist} batch={w.nq} nprobe={NPROBE} R={R}")
    X = database(w)
    Q = queries(w)[:w.nq]
    rng = np.random.default_rng(2024)
    C = np.asarray(X[np.sort(rng.choice(w.n, w.nlist, replace=False))], np.float64)
    T = np.asarray(X[np.sort(rng.choice(w.n, 1 << 17, replace=False))], np.float64)
    for _ in range(2):
        a, dmin = O.assign(T, C)
        C = O.lloyd_update(T, a, C, dmin)
    C32 = C.astype(np.float32)
    P32 = O.random_orthogonal(w.d, rng).astype(np.float32)
    _say("[fullsize] oracle centroids and P ready; building the library index")
    lib = Index.build(X, w.nlist, bq=w.bq, centroids=C32, rotation=P32)
    assign = lib.export("assign").astype(np.int64)
    order = np.argsort(assign, kind="stable")
    starts = np.searchsorted(assign[order], np.arange(w.nlist + 1))
    members = lambda j: order[starts[j]:starts[j + 1]]  # ascending ids
    yield dict(w=w, X=X, Q=Q, C=C32, P=P32, lib=lib, assign=assign, members=members)
    lib.close()


@pytest.fixture(scope="module")
def oracle_pairs(full):
    """The oracle's probes of every batch query and its qu / scalars for every
    (query, probe) pair (FP64 rotation and quantisation)."""
    w, Q, C, P = full["w"], full["Q"], full["C"], full["P"]
    _say("[fullsize] oracle probes and quantised residuals of the batch")
    Cr = C.astype(np.float64) @ P.astype(np.float64)
    probes = np.empty((len(Q), NPROBE), np.int32)
    pdist = np.empty((len(Q), NPROBE))
    qu = np.empty((len(Q), NPROBE, w.d), np.uint8)
    sc = np.empty((len(Q), NPROBE, 3), np.float32)
    terms = []
    for i in range(len(Q)):
        pr, pd = O.probe(Q[i], C, NPROBE)
        probes[i], pdist[i] = pr, pd
        qrot = O.rotate(Q[i], P)
        row = []
        for p, j in enumerate(pr):
            r = qrot - Cr[j]
            u, vl, delta, squ = O.quantize(r, w.bq)
            rn2 = float(r @ r)
            qu[i, p] = u
            sc[i, p] = (rn2, vl, delta)
            if i in SAMPLED:
                row.append((rn2, vl, delta, squ, u))
        terms.append(row)
    return dict(probes=probes, pdist=pdist, qu=qu, sc=sc, terms=terms)


@pytest.fixture(scope="module")
def injected_batch(full, oracle_pairs):
    lib = full["lib"]
    _say("[fullsize] full batch with the oracle's probes, qu and scalars injected")
    lib.set_timing(True)
    out = lib.search_debug(full["Q"], NPROBE, K, R, inject_probes=oracle_pairs["probes"],
                           inject_qu=oracle_pairs["qu"], inject_scalars=oracle_pairs["sc"],
                           want={"cand_ids", "cand_est", "ids", "sqdist"})
    t = lib.timings()
    lib.set_timing(False)
    assert t["group_launches"] > 0  # the list-major scan ran (for the large chunks)
    return out


def _oracle_lists(full, oracle_pairs, i):
    """Oracle estimates of every member of query i's probed lists."""
    X, C, P, w = full["X"], full["C"], full["P"], full["w"]
    out = []
    for p, j in enumerate(oracle_pairs["probes"][i]):
        ids = full["members"](int(j))
        rn2, vl, delta, squ, u = oracle_pairs["terms"][i][p]
        codes, n_x, alpha = O.encode(X[ids], C, np.full(len(ids), j), P)
        E, ip, pop = O.est_terms(codes, u, vl, delta, w.d)
        est = O.estimate(rn2, E, n_x, alpha, w.d)
        S = est_scale(rn2, vl, delta, squ, ip, pop, n_x, alpha, w.d)
        out.append(dict(ids=ids, ip=ip, est=est, S=S))
    return out


@pytest.fixture(scope="module")
def sampled_oracle(full, oracle_pairs):
    _say("[fullsize] oracle encoding and estimates of the sampled queries' probed lists")
    return {i: _oracle_lists(full, oracle_pairs, i) for i in SAMPLED}


def test_probes_match_oracle(full, oracle_pairs):
    lib, C, Q, d = full["lib"], full["C"], full["Q"], full["w"].d
    got = lib.search_debug(Q, NPROBE, K, R, want={"probes"})["probes"]
    cn = np.sum(C.astype(np.float64) ** 2, axis=1)
    for i in range(len(Q)):
        if np.array_equal(got[i], oracle_pairs["probes"][i]):
            continue
        # only near-ties of the FP32 probe score may reorder or swap lists
        pd = {int(j): v for j, v in zip(oracle_pairs["probes"][i], oracle_pairs["pdist"][i])}
        dist = lambda j: pd[j] if j in pd else float(np.sum((C[j].astype(np.float64) - Q[i]) ** 2))
        tol = lambda j: 4 * d * 2.0 ** -24 * (cn[j] + 2 * math.sqrt(cn[j]) * float(np.linalg.norm(Q[i]))) + 1e-6
        bad = set_diff_ok(got[i], oracle_pairs["probes"][i], dist, oracle_pairs["pdist"][i][-1], tol)
        assert not bad, (i, bad[:5])


def test_membership_sound(full, oracle_pairs):
    X, C, assign = full["X"], full["C"], full["assign"]
    assert np.bincount(assign, minlength=full["w"].nlist).sum() == full["w"].n
    rng = np.random.default_rng(5)
    for i in SAMPLED:
        for j in rng.choice(oracle_pairs["probes"][i], 16, replace=False):
            ids = full["members"](int(j))
            a, dmin = O.assign(X[ids], C)
            wrong = ids[a != j]
            for v in wrong:  # allowed only at an FP32-level tie with list j
                dj = float(np.sum((X[v].astype(np.float64) - C[j]) ** 2))
                assert dj - dmin[np.searchsorted(ids, v)] <= 1e-5 * dj, (j, v)


@pytest.mark.parametrize("scan,group", [(1, 0), (2, 32), (2, 64)],
                         ids=["popcount", "list-major-G32", "list-major-G64"])
def test_p4_p5_sampled_queries(full, oracle_pairs, sampled_oracle, scan, group):
    """Every estimate of the sampled queries' 512 probed lists, formed by the
    popcount scan or by the list-major scan in the benchmark's item size (32
    queries, two matrix-core tiles) and in the four-tile form."""
    lib, Q = full["lib"], full["Q"]
    rows = list(SAMPLED)
    lib.set_option("scan", scan)
    lib.set_option("group_size", group)
    lib.set_timing(True)
    try:
        out = lib.search_debug(Q[rows], NPROBE, K, R, inject_probes=oracle_pairs["probes"][rows],
                               inject_qu=oracle_pairs["qu"][rows], inject_scalars=oracle_pairs["sc"][rows],
                               want={"ip", "est"})
        t = lib.timings()
    finally:
        lib.set_timing(False)
        lib.set_option("scan", 0)
        lib.set_option("group_size", 0)
    if scan == 2:
        assert t["group_launches"] > 0 and t["popc_launches"] == 0, t
    else:
        assert t["group_launches"] == 0, t
    worst = 0.0
    for t, i in enumerate(rows):
        for p, ol in enumerate(sampled_oracle[i]):
            m = len(ol["ids"])
            np.testing.assert_array_equal(out["ip"][t, p, :m], ol["ip"], err_msg=f"q{i} p{p}")
            err = np.abs(out["est"][t, p, :m].astype(np.float64) - ol["est"]) / ol["S"]
            if m:
                worst = max(worst, float(err.max()))
            assert np.all(err <= 1e-5), (i, p, float(err.max()))
    _say(f"[fullsize] scan {scan} G {group}: P4 exact, P5 worst scaled error {worst:.2e}")


def test_p6_p7_sampled_queries_in_batch(full, injected_batch, sampled_oracle):
    X, Q = full["X"], full["Q"]
    out = injected_batch
    for i in SAMPLED:
        ids = np.concatenate([ol["ids"] for ol in sampled_oracle[i]])
        est = np.concatenate([ol["est"] for ol in sampled_oracle[i]])
        S = np.concatenate([ol["S"] for ol in sampled_oracle[i]])
        val = dict(zip(ids.tolist(), est.tolist()))
        tol = dict(zip(ids.tolist(), (2e-5 * S).tolist()))
        ref_v, ref_i = O.topk_lex(est, ids, R)
        boundary = ref_v[-1]
        bad = set_diff_ok(out["cand_ids"][i], ref_i, lambda x: val[x], boundary, lambda x: tol[x])
        assert not bad, ("P6", i, bad[:5])
        # every returned candidate's estimate within 1e-5 S of the oracle's
        for x, e in zip(out["cand_ids"][i].tolist(), out["cand_est"][i].tolist()):
            if x >= 0:
                assert abs(e - val[x]) <= 0.5 * tol[x], ("P5 of a candidate", i, x, e, val[x])
        # P7: final top-k from the oracle's candidates
        fv, fi = O.rerank(Q[i], X, ref_i, K)
        exact = lambda x: float(np.sum((X[x].astype(np.float64) - Q[i].astype(np.float64)) ** 2))

        def tol7(x):
            if x in val and abs(val[x] - boundary) <= tol[x]:
                return math.inf  # a P6 near-tie at the candidate boundary
            return 1e-5 * max(exact(x), fv[-1]) + 1e-6
        bad = set_diff_ok(out["ids"][i], fi, exact, fv[-1], tol7)
        assert not bad, ("P7", i, bad[:5])


def test_batch_results_exact_and_scan_forms_agree(full):
    lib, X, Q = full["lib"], full["X"], full["Q"]
    want = {"cand_ids", "cand_est", "ids", "sqdist"}
    _say("[fullsize] un-injected batch: list-major vs query-major")
    outs = {}
    for scan in (2, 1):
        lib.set_option("scan", scan)
        try:
            outs[scan] = lib.search_debug(Q, NPROBE, K, R, want=want)
        finally:
            lib.set_option("scan", 0)
    for key in want:
        np.testing.assert_array_equal(outs[2][key], outs[1][key], err_msg=key)
    ids, dd = outs[2]["ids"], outs[2]["sqdist"]
    assert np.all(ids >= 0)
    for i in range(len(Q)):
        assert len(set(ids[i].tolist())) == K
        assert np.all(np.diff(dd[i]) >= 0)
    diff = X[ids].astype(np.float64) - Q[:, None, :].astype(np.float64)
    ex = np.sum(diff * diff, axis=2)
    assert np.all(np.abs(dd - ex) <= 4 * X.shape[1] * 2.0 ** -24 * ex + 1e-30)
