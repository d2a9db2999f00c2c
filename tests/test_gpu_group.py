"""GPU tests of the list-major matrix-core scan (fp4 x fp8 for B_q <= 4, int8
above).

Its estimator epilogue is the same expression as the query-major popcount
scan's and the selection is exact, so both scans must return identical
candidates and results; with the oracle's probes, qu and scalars injected the
candidates must also match the oracle's (same rule as test_gpu_parity P6).
A tiny pool capacity forces the overflow path (the flagged queries are
searched again from scratch by the fused query-major scan).
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import est_scale, lib_index, make_case, set_diff_ok

pytestmark = pytest.mark.gpu

WANT = {"cand_ids", "cand_est", "ids", "sqdist"}

SHAPES = [
    # name, n, d, nlist, nq, nprobe, k, R, kind, bq
    ("g128", 20_000, 128, 16, 150, 12, 10, 100, "mixture", 4),
    ("g96", 12_000, 96, 12, 70, 9, 10, 60, "unit_mixture", 4),
    ("g40_bq8", 9_000, 40, 10, 90, 7, 5, 40, "mixture", 8),
    ("g13", 4_000, 13, 8, 33, 6, 5, 30, "mixture", 2),
    ("g256", 6_000, 256, 8, 40, 5, 10, 80, "gamma_int", 4),
    # the three ways qu enters the signed-byte MFMA: doubled (B_q <= 6),
    # plain (B_q = 7), offset by -128 (B_q = 8, above)
    ("g72_bq6", 8_000, 72, 10, 80, 6, 5, 40, "mixture", 6),
    ("g64_bq7", 8_000, 64, 10, 80, 6, 5, 40, "mixture", 7),
    # the fp4 x fp8 form (B_q <= 4) at its edges: a second 128-dimension step
    # padded past d = 200, and the smallest query codes (2 qu <= 14, <= 2)
    ("g200_bq3", 6_000, 200, 8, 40, 5, 10, 80, "mixture", 3),
    ("g160_bq1", 6_000, 160, 8, 40, 5, 10, 80, "unit_mixture", 1),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=list(enumerate(SHAPES)), ids=[s[0] for s in SHAPES])
def gcase(request):
    seed, (name, n, d, nlist, nq, nprobe, k, R, kind, bq) = request.param
    _say(f"[group {name}] n={n} d={d} nlist={nlist} nq={nq} nprobe={nprobe} R={R} bq={bq}")
    X, Q, idx = make_case(n, d, nlist, nq, seed=100 + seed, kind=kind)
    idx.bq = bq
    lib = lib_index(X, idx, bq=bq)
    return dict(name=name, X=X, Q=Q, idx=idx, lib=lib, nprobe=nprobe, k=k, R=R, d=d)


def _run(lib, Q, nprobe, k, R, scan, pool_cap=0, lm_only=False, want_extra=(), **kw):
    """lm_only: the list-major scan produced every result itself (scan 2 with
    no pool overflow, so no query was redone by the query-major scan)."""
    lib.set_option("scan", scan)
    lib.set_option("pool_cap", pool_cap)
    if lm_only:
        lib.set_timing(True)
    try:
        out = lib.search_debug(Q, nprobe, k, R, want=WANT | set(want_extra), **kw)
        if lm_only:
            t = lib.timings()
            assert t["group_launches"] > 0 and t["popc_launches"] == 0, t
        return out
    finally:
        if lm_only:
            lib.set_timing(False)
        lib.set_option("scan", 0)
        lib.set_option("pool_cap", 0)


def test_group_equals_query_major(gcase):
    lib, Q = gcase["lib"], gcase["Q"]
    a = _run(lib, Q, gcase["nprobe"], gcase["k"], gcase["R"], scan=1)
    b = _run(lib, Q, gcase["nprobe"], gcase["k"], gcase["R"], scan=2, lm_only=True)
    for key in WANT:
        np.testing.assert_array_equal(b[key], a[key], err_msg=key)


@pytest.mark.parametrize("cap", [1, 37])
def test_group_overflow_path_is_exact(gcase, cap):
    lib, Q = gcase["lib"], gcase["Q"]
    a = _run(lib, Q, gcase["nprobe"], gcase["k"], gcase["R"], scan=1)
    b = _run(lib, Q, gcase["nprobe"], gcase["k"], gcase["R"], scan=2, pool_cap=cap)
    for key in WANT:
        np.testing.assert_array_equal(b[key], a[key], err_msg=f"{key} cap {cap}")


def test_group_candidates_match_oracle(gcase):
    """Oracle probes, qu and scalars injected; every chunk on the list-major
    scan, which also writes out each estimate it forms. P4: its integer inner
    products equal the oracle's for every (query, vector); P5: its d_hat^2 is
    within 1e-5 S of the oracle's. P6: candidate sets equal up to near-ties at
    the R-th value (an element and the boundary may each move by 1e-5 S, so
    sets are compared with a 2e-5 S window), and every returned candidate's
    estimate within 1e-5 S of the oracle's."""
    lib, Q, X, idx = gcase["lib"], gcase["Q"], gcase["X"], gcase["idx"]
    nprobe, k, R, d = gcase["nprobe"], gcase["k"], gcase["R"], gcase["d"]
    _, _, st = O.search(idx, X, Q, nprobe, k, R, stages=True)
    nq = len(Q)
    probes = np.array(st["probes"], np.int32)
    qu = np.zeros((nq, nprobe, d), np.uint8)
    sc = np.zeros((nq, nprobe, 3), np.float32)
    for qi in range(nq):
        for p in range(nprobe):
            qu[qi, p] = st["qu"][qi][p]
            sc[qi, p] = (st["rnorm2"][qi][p], st["vl"][qi][p], st["delta"][qi][p])
    out = _run(lib, Q, nprobe, k, R, scan=2, lm_only=True, inject_probes=probes, inject_qu=qu,
               inject_scalars=sc)
    dumps = _run(lib, Q, nprobe, k, R, scan=2, lm_only=True, inject_probes=probes, inject_qu=qu,
                 inject_scalars=sc, want_extra={"ip", "est"})
    worst = 0.0
    for qi in range(nq):
        val, tol = {}, {}
        for p, pl in enumerate(st["per_list"][qi]):
            S = est_scale(st["rnorm2"][qi][p], st["vl"][qi][p], st["delta"][qi][p],
                          st["sumqu"][qi][p], pl["ip"], pl["pop"], idx.n_x[pl["ids"]],
                          idx.alpha[pl["ids"]], d)
            m = len(pl["ids"])
            np.testing.assert_array_equal(dumps["ip"][qi, p, :m], pl["ip"], err_msg=f"P4 q{qi} p{p}")
            err = np.abs(dumps["est"][qi, p, :m].astype(np.float64) - pl["est"]) / S
            assert np.all(err <= 1e-5), (qi, p, float(err.max()))
            worst = max(worst, float(err.max()) if m else 0.0)
            for i, e, s in zip(pl["ids"].tolist(), pl["est"].tolist(), S.tolist()):
                val[i], tol[i] = e, s
        ref = st["cand_ids"][qi]
        rv = ref[ref >= 0]
        boundary = val[int(rv[-1])] if len(rv) else math.inf
        bad = set_diff_ok(out["cand_ids"][qi], ref, lambda x: val[x], boundary, lambda x: 2e-5 * tol[x])
        assert not bad, (qi, bad[:5])
        g = out["cand_ids"][qi]
        for i, e in zip(g[g >= 0].tolist(), out["cand_est"][qi].tolist()):
            assert abs(e - val[i]) <= 1e-5 * tol[i]
        np.testing.assert_array_equal(out["cand_ids"][qi], dumps["cand_ids"][qi])
    _say(f"[group {gcase['name']}] P4 exact, P5 worst {worst:.2e} S")


@pytest.mark.parametrize("block", [1, 2, 16])
def test_group_index_blocks_invariant(gcase, block):
    """Items over index blocks of `block` micro-blocks (a long list shared out
    over several workgroups, Sec. 3.3.1): candidates and results equal the
    query-major scan's, and every estimate written out equals that of
    whole-list items (each vector's dump lands at its position in its list)."""
    lib, Q = gcase["lib"], gcase["Q"]
    nprobe, k, R = gcase["nprobe"], gcase["k"], gcase["R"]
    a = _run(lib, Q, nprobe, k, R, scan=1)
    lib.set_option("block", block)
    try:
        b = _run(lib, Q, nprobe, k, R, scan=2, lm_only=True, want_extra={"ip", "est"})
    finally:
        lib.set_option("block", -1)
    for key in WANT:
        np.testing.assert_array_equal(b[key], a[key], err_msg=f"{key} block {block}")
    lib.set_option("block", 0)
    try:
        c = _run(lib, Q, nprobe, k, R, scan=2, lm_only=True, want_extra={"ip", "est"})
    finally:
        lib.set_option("block", -1)
    np.testing.assert_array_equal(b["ip"], c["ip"])
    np.testing.assert_array_equal(b["est"], c["est"])


def test_fused_buffer_shrinks_mid_chunk():
    """Lists of ~10k vectors: the first fused chunk holds more candidates than
    the fused kernel's LDS buffer, so it keeps only the best R and lowers the
    threshold several times while it scans. Results equal the query-major
    scan's."""
    _say("[group] fused chunk larger than its buffer: n=640000 d=32 nlist=64 nq=160")
    X, Q, idx = make_case(640_000, 32, 64, 160, seed=141)
    lib = lib_index(X, idx)
    try:
        lib.set_timing(True)
        b = _run(lib, Q, 16, 10, 200, scan=0)
        t = lib.timings()
        lib.set_timing(False)
        assert t["popc_launches"] > 0, t  # the fused chunk ran
        a = _run(lib, Q, 16, 10, 200, scan=1)
        for key in WANT:
            np.testing.assert_array_equal(b[key], a[key], err_msg=key)
    finally:
        lib.close()


def test_fused_and_list_major_chunks_agree():
    """A batch large enough (>= 128 queries) with lists shared by few queries in
    the first chunks: those chunks take the fused one-workgroup-per-query scan,
    the later ones the list-major scan. Results equal the query-major scan's,
    also for a mixed batch (per-query nprobe / k / rerank_n)."""
    _say("[group] schedule with fused query-major chunks: n=40000 d=128 nlist=256 nq=300")
    X, Q, idx = make_case(40_000, 128, 256, 300, seed=140)
    lib = lib_index(X, idx)
    try:
        lib.set_timing(True)
        b = _run(lib, Q, 64, 10, 200, scan=0)
        t = lib.timings()
        lib.set_timing(False)
        assert t["popc_launches"] > 0 and t["group_launches"] > 0, t
        a = _run(lib, Q, 64, 10, 200, scan=1)
        for key in WANT:
            np.testing.assert_array_equal(b[key], a[key], err_msg=key)
        rng = np.random.default_rng(9)
        npb = rng.integers(1, 65, len(Q)).astype(np.int32)
        k = rng.choice([1, 10, 25], len(Q)).astype(np.int32)
        R = np.maximum(k, rng.choice([30, 200, 300], len(Q))).astype(np.int32)
        m_ids, m_d = lib.search_mixed(Q, npb, k, R)
        for i in range(0, len(Q), 5):
            x, y = lib.search(Q[i:i + 1], int(npb[i]), int(k[i]), int(R[i]))
            np.testing.assert_array_equal(m_ids[i, :k[i]], x[0])
            np.testing.assert_array_equal(m_d[i, :k[i]], y[0])
    finally:
        lib.close()
