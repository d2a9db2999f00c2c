"""GPU tests of the IVF-Flat scan (RBQ_OPT_ESTIMATOR 2 on an index built with
ivf_flat), the comparison system of Sec. 4.2: exact distances of the
full-precision vectors of the probed lists on the FP32 matrix cores,
||q||^2 + ||x||^2 - 2 <q, x>, the best rerank_n re-ranked exactly.

Against the oracle's IVF-Flat search (FP64 brute force over the probed lists),
with the oracle's centroids and assignment in the library index:
  * final ids equal up to exact-distance near-ties: an element may swap with
    the k-th only if their FP64 distances differ by less than the FP32 error
    of the product form, 4 (D + 4) 2^-24 (||q||^2 + ||x||^2);
  * returned distances are the exact ones to 4 D 2^-24 relative (the re-rank's
    direct differences);
  * a mixed batch returns each query's result bit for bit as alone;
  * a candidate pool that cannot hold a chunk's survivors fails the search
    (RBQ_ENOMEM) instead of returning a wrong result.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_16007_amd import Index, rbq
from tests._parity import make_case, set_diff_ok

pytestmark = pytest.mark.gpu

U = 2.0 ** -24

SHAPES = [
    # name, n, d, nlist, nq, nprobe, kind
    ("f128", 20_000, 128, 16, 300, 6, "mixture"),
    ("f96", 12_000, 96, 12, 200, 5, "unit_mixture"),
    ("f13", 4_000, 13, 8, 150, 4, "mixture"),
    ("f200", 6_000, 200, 8, 120, 4, "gamma_int"),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=SHAPES, ids=[s[0] for s in SHAPES])
def fcase(request):
    name, n, d, nlist, nq, nprobe, kind = request.param
    _say(f"[ivf-flat {name}] n={n} d={d} nlist={nlist} nq={nq} nprobe={nprobe}")
    X, Q, idx = make_case(n, d, nlist, nq, seed=500 + d, kind=kind)
    lib = Index.build(X, nlist, centroids=idx.centroids, rotation=idx.P,
                      assignment=idx.assign.astype(np.int32), ivf_flat=True, vectors_on_host=False)
    lib.set_option("estimator", 2)
    yield dict(name=name, X=X, Q=Q, idx=idx, lib=lib, nprobe=nprobe, d=d)
    lib.close()


@pytest.mark.parametrize("k,R", [(10, 10), (10, 60), (1, 1)])
def test_ivf_flat_matches_oracle(fcase, k, R):
    lib, Q, X, idx, d = fcase["lib"], fcase["Q"], fcase["X"], fcase["idx"], fcase["d"]
    nprobe = fcase["nprobe"]
    ref_ids, ref_d = O.ivf_flat_search(idx, X, Q, nprobe, k)
    lib.set_timing(True)
    ids, dd = lib.search(Q, nprobe, k, R)
    t = lib.timings()
    lib.set_timing(False)
    assert t["group_launches"] > 0 and t["popc_launches"] == 0, t
    X64, Q64 = X.astype(np.float64), Q.astype(np.float64)
    xn = np.sum(X64 * X64, axis=1)
    for qi in range(len(Q)):
        exact = lambda x: float(np.sum((X64[x] - Q64[qi]) ** 2))
        qn = float(Q64[qi] @ Q64[qi])
        tol = lambda x: 4 * (d + 4) * U * (qn + xn[x]) + 1e-6
        bad = set_diff_ok(ids[qi], ref_ids[qi], exact, ref_d[qi][-1], tol)
        assert not bad, (qi, bad[:5])
        for x, v in zip(ids[qi].tolist(), dd[qi].tolist()):
            assert x >= 0
            e = exact(x)
            assert abs(v - e) <= 4 * d * U * e + 1e-30
        assert np.all(np.diff(dd[qi]) >= 0)


def test_ivf_flat_mixed_equals_alone(fcase):
    lib, Q = fcase["lib"], fcase["Q"]
    rng = np.random.default_rng(6)
    nq = len(Q)
    npb = rng.integers(1, fcase["nprobe"] + 1, nq).astype(np.int32)
    k = rng.choice([1, 5, 10], nq).astype(np.int32)
    R = np.maximum(k, rng.choice([10, 40], nq)).astype(np.int32)
    m_ids, m_d = lib.search_mixed(Q, npb, k, R)
    for i in range(0, nq, 7):
        a, b = lib.search(Q[i:i + 1], int(npb[i]), int(k[i]), int(R[i]))
        np.testing.assert_array_equal(m_ids[i, :k[i]], a[0])
        np.testing.assert_array_equal(m_d[i, :k[i]], b[0])


def test_ivf_flat_pool_overflow_fails(fcase):
    lib, Q = fcase["lib"], fcase["Q"]
    lib.set_option("pool_cap", 3)
    try:
        with pytest.raises(rbq.RbqError) as e:
            lib.search(Q[:50], fcase["nprobe"], 10, 10)
        assert e.value.status == rbq.RBQ_ENOMEM and "overflowed" in str(e.value)
    finally:
        lib.set_option("pool_cap", 0)
    ids, _ = lib.search(Q[:50], fcase["nprobe"], 10, 10)  # usable afterwards
    assert np.all(ids >= 0)
