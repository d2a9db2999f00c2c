"""GPU tests of the unquantised-query estimator (RBQ_OPT_ESTIMATOR 1): the
rotated residual r = P^T q - P^T c stays FP32 and E = sum_d b_d r_d comes from
sign-pattern tables of 8-dimension groups (4 when d > 128), as the paper's
accelerator path evaluates Eq. rabitq-ip-estimator without query quantisation
(Sec. 4.3).

Against the oracle's unquantised search (est_terms_unquantized), with the
oracle's probes and FP64 rotated queries (rounded to FP32) injected:
  * every estimate of every probed list within 1e-5 S, with S the sum of the
    magnitudes of the estimator's terms:
        S = ||r||^2 + n_x^2 + 2 n_x (sum_d |r_d|) / (sqrt(D) alpha)
    (the GPU forms r from FP32-rounded rotated vectors: |dr_d| <= u (|P^T q|_d
    + |P^T c|_d + |r_d|), and sums at most 2 D / 8 + D terms in FP32);
  * candidate sets (P6: sets equal up to a 2e-5 S window at the R-th value,
    each returned estimate within 1e-5 S) and final ids (P7);
  * a mixed batch returns each query's result bit for bit as alone.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import lib_index, make_case, set_diff_ok

pytestmark = pytest.mark.gpu

SHAPES = [
    # name, n, d, nlist, nq, nprobe, k, R, kind
    ("u128", 20_000, 128, 16, 60, 6, 10, 100, "mixture"),
    ("u96", 12_000, 96, 12, 50, 5, 10, 60, "unit_mixture"),
    ("u13", 4_000, 13, 8, 33, 4, 5, 30, "mixture"),
    ("u200", 6_000, 200, 8, 30, 4, 10, 80, "gamma_int"),
    ("u960", 3_000, 960, 6, 20, 3, 10, 50, "blocks_abs"),
]


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", params=SHAPES, ids=[s[0] for s in SHAPES])
def ucase(request):
    name, n, d, nlist, nq, nprobe, k, R, kind = request.param
    _say(f"[unquantised {name}] n={n} d={d} nlist={nlist} nq={nq} nprobe={nprobe} R={R}")
    X, Q, idx = make_case(n, d, nlist, nq, seed=300 + d, kind=kind)
    lib = lib_index(X, idx)
    lib.set_option("estimator", 1)
    yield dict(name=name, X=X, Q=Q, idx=idx, lib=lib, nprobe=nprobe, k=k, R=R, d=d)
    lib.close()


def _scale(rn2, r, n_x, alpha, d):
    n_x = np.asarray(n_x, np.float64)
    return rn2 + n_x * n_x + 2 * n_x * float(np.sum(np.abs(r))) / (math.sqrt(d) * np.asarray(alpha, np.float64))


def test_unquantized_matches_oracle(ucase):
    lib, Q, X, idx = ucase["lib"], ucase["Q"], ucase["X"], ucase["idx"]
    nprobe, k, R, d = ucase["nprobe"], ucase["k"], ucase["R"], ucase["d"]
    ref_ids, ref_d, st = O.search(idx, X, Q, nprobe, k, R, stages=True, unquantized=True)
    probes = np.array(st["probes"], np.int32)
    qrot = np.array(st["qrot"], np.float64).astype(np.float32)
    out = lib.search_debug(Q, nprobe, k, R, inject_probes=probes, inject_qrot=qrot,
                           want={"est", "cand_ids", "cand_est", "ids", "sqdist"})
    worst = 0.0
    for qi in range(len(Q)):
        val, tol = {}, {}
        for p, pl in enumerate(st["per_list"][qi]):
            m = len(pl["ids"])
            S = _scale(st["rnorm2"][qi][p], pl["r"], idx.n_x[pl["ids"]], idx.alpha[pl["ids"]], d)
            err = np.abs(out["est"][qi, p, :m].astype(np.float64) - pl["est"]) / S
            assert np.all(err <= 1e-5), (qi, p, float(err.max()))
            worst = max(worst, float(err.max()) if m else 0.0)
            for i, e, s in zip(pl["ids"].tolist(), pl["est"].tolist(), S.tolist()):
                val[i], tol[i] = e, s
        ref = st["cand_ids"][qi]
        rv = ref[ref >= 0]
        boundary = val[int(rv[-1])] if len(rv) else math.inf
        bad = set_diff_ok(out["cand_ids"][qi], ref, lambda x: val[x], boundary, lambda x: 2e-5 * tol[x])
        assert not bad, ("P6", qi, bad[:5])
        for x, e in zip(out["cand_ids"][qi].tolist(), out["cand_est"][qi].tolist()):
            if x >= 0:
                assert abs(e - val[x]) <= 1e-5 * tol[x], ("P5 of a candidate", qi, x)
        exact = lambda x: float(np.sum((X[x].astype(np.float64) - Q[qi].astype(np.float64)) ** 2))
        fb = ref_d[qi][-1]

        def tol7(x):
            if x in val and abs(val[x] - boundary) <= 2e-5 * tol[x]:
                return math.inf  # a P6 near-tie at the candidate boundary
            return 1e-5 * max(exact(x), fb) + 1e-6
        bad = set_diff_ok(out["ids"][qi], ref_ids[qi], exact, fb, tol7)
        assert not bad, ("P7", qi, bad[:5])
    _say(f"[unquantised {ucase['name']}] P5 worst {worst:.2e} S")


def test_unquantized_mixed_equals_alone(ucase):
    lib, Q = ucase["lib"], ucase["Q"]
    rng = np.random.default_rng(4)
    nq = len(Q)
    npb = rng.integers(1, ucase["nprobe"] + 1, nq).astype(np.int32)
    k = rng.choice([1, 5, ucase["k"]], nq).astype(np.int32)
    R = np.maximum(k, rng.choice([5, ucase["R"]], nq)).astype(np.int32)
    m_ids, m_d = lib.search_mixed(Q, npb, k, R)
    for i in range(0, nq, 3):
        a, b = lib.search(Q[i:i + 1], int(npb[i]), int(k[i]), int(R[i]))
        np.testing.assert_array_equal(m_ids[i, :k[i]], a[0])
        np.testing.assert_array_equal(m_d[i, :k[i]], b[0])
