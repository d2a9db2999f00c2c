"""The library's GPU k-means (Sec. 3.1.1 Phases 1-2) against the oracle's
procedure with the library's reading of the seeding (k-means++ over the evenly
strided subset of at most 32 nlist training rows, ``seed_rows``), and with
random initial centroids (``init="random"``, Sec. 3.1.1 Phase 1).

The two draw their random numbers from different generators, so they are
compared where the outcome does not depend on the draws or only slightly:
  * well-separated clusters: both return the true centres (to the noise), in
    some order;
  * a mixture without clear separation: the objectives (sum of squared
    distances to the nearest centroid, FP64) agree within 3%;
  * converged centroids are the means of their points (a Lloyd fixed point).
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2605_16007_amd import Index

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _objective(X, C):
    _, dmin = O.assign(X, C)
    return float(dmin.sum())


def test_kmeans_separated_clusters():
    _say("[kmeans] separated clusters n=4000 d=16 nlist=8")
    rng = np.random.default_rng(11)
    centres = np.eye(16)[:8] * 100.0
    X = (centres[rng.integers(0, 8, 4000)] + 0.05 * rng.normal(size=(4000, 16))).astype(np.float32)
    lib = Index.build(X, 8, seed=3)
    try:
        Cl = lib.export("centroids").astype(np.float64)
    finally:
        lib.close()
    Co = O.kmeans(X, 8, np.random.default_rng(3), seed_rows=32 * 8)
    for C in (Cl, Co):
        d = O.sqdist(C, centres)
        assert np.all(np.min(d, axis=1) < 0.01)
        assert len(set(np.argmin(d, axis=1))) == 8
    d = O.sqdist(Cl, Co)
    assert np.all(np.min(d, axis=1) < 1e-6 * 100.0 ** 2)


@pytest.mark.parametrize("seed,init", [(0, "kmeans++"), (1, "kmeans++"), (2, "random")])
def test_kmeans_objective_matches_oracle(seed, init):
    from synth import database, get
    w = get("mixture128", n=20_000, d=32, nlist=64, centres=128, seed=seed)
    _say(f"[kmeans] mixture n={w.n} d={w.d} nlist={w.nlist} seed={seed} init={init}")
    X = database(w)
    lib = Index.build(X, w.nlist, seed=seed, kmeans_init=init)
    try:
        Cl = lib.export("centroids").astype(np.float64)
        a = lib.export("assign")
    finally:
        lib.close()
    Co = O.kmeans(X, w.nlist, np.random.default_rng(seed), seed_rows=32 * w.nlist, init=init)
    ol, oo = _objective(X, Cl), _objective(X, Co)
    _say(f"[kmeans] objective library {ol:.1f}, oracle {oo:.1f} (ratio {ol / oo:.4f})")
    assert 0.97 <= ol / oo <= 1.03
    # the library's assignment is the nearest centroid (ties within FP32 error)
    ao, dmin = O.assign(X, Cl)
    wrong = np.flatnonzero(a != ao)
    for i in wrong:
        di = float(np.sum((X[i].astype(np.float64) - Cl[a[i]]) ** 2))
        assert di - dmin[i] <= 1e-5 * max(di, 1e-30)


def test_kmeans_converged_centroids_are_means():
    from synth import database, get
    w = get("mixture128", n=6_000, d=16, nlist=12, centres=12, seed=4)
    X = database(w)
    # (every row trains, so the fixed point is over all of them)
    lib = Index.build(X, w.nlist, seed=4, kmeans_iters=200, kmeans_restarts=1, train_n=w.n)
    try:
        C = lib.export("centroids").astype(np.float64)
    finally:
        lib.close()
    a, _ = O.assign(X, C)
    for j in range(w.nlist):
        m = a == j
        assert m.any()
        mean = X[m].astype(np.float64).mean(axis=0)
        assert np.max(np.abs(C[j] - mean)) <= 1e-4 * (1.0 + np.max(np.abs(mean)))
