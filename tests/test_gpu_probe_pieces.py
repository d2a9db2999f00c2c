"""Probe selection for more lists than one register-resident row holds
(nlist > 8192, as at 400M x 96 with 65,536 lists): the first 2048 scores
(nprobe <= 256) or 8192 of a query's row set a bound that the rest of the row
streams past, the keys below it being cut back to the nprobe best whenever
they might overflow. Checked against the oracle's FP64 probe ranking (lists
whose exact distances lie within FP32 rounding of the boundary may swap),
with a ragged last tile, nprobe on both sides of 256 and up to 4000, and
lists ordered far-to-near (every later score passes a loose first bound, so
the cut-back runs many times per row)."""
import math
import sys

import numpy as np
import pytest

import oracle as O
from tests._parity import set_diff_ok

pytestmark = pytest.mark.gpu

D, NQ = 96, 300


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nlist,nprobe,order", [(20_000, 128, "random"), (20_000, 4000, "random"),
                                                (65_536, 128, "random"), (65_536, 1000, "random"),
                                                (20_000, 128, "far_first"), (20_000, 4000, "far_first"),
                                                (65_536, 256, "far_first"), (20_000, 257, "random")])
def test_probes_over_pieces(nlist, nprobe, order):
    from synth import database, get, queries
    from paper_2605_16007_amd import Index
    n = nlist + 5000
    w = get("unit96_400m", n=n, nlist=nlist, nq=NQ, centres=4096)
    _say(f"[probe pieces] n={n} d={D} nlist={nlist} nprobe={nprobe} order={order} queries={NQ}")
    X = database(w)
    Q = queries(w)
    rng = np.random.default_rng(nlist + nprobe)
    C = np.asarray(X[np.sort(rng.choice(n, nlist, replace=False))], np.float32)
    if order == "far_first":  # descending distance to the mean query
        far = np.sum((C.astype(np.float64) - Q.astype(np.float64).mean(axis=0)) ** 2, axis=1)
        C = np.ascontiguousarray(C[np.argsort(-far, kind="stable")])
    ix = Index.build(X, nlist, centroids=C, vectors_on_host=False)
    try:
        got = ix.search_debug(Q, nprobe, 10, 100, want={"probes"})["probes"]
    finally:
        ix.close()
    assert got.shape == (NQ, nprobe)
    cn = np.sum(C.astype(np.float64) ** 2, axis=1)
    mism = 0
    for i in range(NQ):
        assert len(set(got[i].tolist())) == nprobe and got[i].min() >= 0 and got[i].max() < nlist
        pr, pd = O.probe(Q[i], C, nprobe)
        if np.array_equal(got[i], pr):
            continue
        mism += 1
        dist = lambda j: float(np.sum((C[j].astype(np.float64) - Q[i]) ** 2))
        tol = lambda j: 4 * D * 2.0 ** -24 * (cn[j] + 2 * math.sqrt(cn[j]) * float(np.linalg.norm(Q[i]))) + 1e-6
        bad = set_diff_ok(got[i], pr, dist, pd[-1], tol)
        assert not bad, (i, bad[:5])
        # the returned order ascends in distance, up to FP32 rounding
        gd = [dist(int(j)) for j in got[i]]
        for t in range(nprobe - 1):
            a, b = int(got[i][t]), int(got[i][t + 1])
            assert gd[t + 1] >= gd[t] - tol(a) - tol(b), (i, t, a, b)
    _say(f"[probe pieces] {NQ - mism} of {NQ} queries identical to the oracle, the rest differ at near-ties")
