"""Helpers for GPU-vs-oracle parity: shared fixtures, tolerance rules.

Tolerance rules (derived from FP32 arithmetic; unit roundoff u = 2^-24):
  * codes: bit-exact, except a dimension whose FP64 rotated residual lies within
    tau = 4 D u n_x of zero (the encoder runs in FP64, so none are expected);
  * factors n_x, alpha: 2e-7 relative (both sides round an FP64 value to FP32);
  * qu: equal, except a dimension whose oracle y = (r - v_l)/Delta lies within
    eta of a rounding boundary, where eta bounds the FP32 error of the GPU's
    rotated residual; such dimensions may differ by exactly 1;
  * integer inner products (oracle qu injected): bit-exact;
  * d_hat^2 (oracle qu and scalars injected): |diff| <= 1e-5 * S, with S the sum
    of the magnitudes of the estimator's terms:
        S = ||r||^2 + n_x^2 + 2 n_x (|v_l| |2 pop - D| + Delta |2 ip - sum qu|) / (sqrt(D) alpha)
    (d_hat^2 itself can be near zero or negative, so a plain relative bound
    would be meaningless there);
  * candidate / final ids: equal as sets, except elements whose oracle value
    lies within the tolerance of the boundary (R-th or k-th) value.
"""
from __future__ import annotations

import math

import numpy as np

import oracle as O

U32 = 2.0 ** -24


def make_case(n, d, nlist, nq, seed=0, kind="mixture", kmeans_iters=6):
    """Synthetic data, oracle centroids / P / assignment, and the oracle index."""
    from synth import get, database, queries
    base = {"mixture": "mixture128", "gamma_int": "sift10m", "blocks_abs": "embed960",
            "unit_mixture": "unit96_400m"}[kind]
    extra = {}
    if kind in ("mixture", "unit_mixture"):
        extra = {"centres": max(8, nlist // 2)}
    w = get(base, n=n, d=d, nlist=nlist, nq=nq, seed=seed, **extra)
    X = database(w)
    Q = queries(w)
    rng = np.random.default_rng(1000 + seed)
    C = O.kmeans(X, nlist, rng, iters=kmeans_iters, restarts=1).astype(np.float32)
    P = O.random_orthogonal(d, rng).astype(np.float32)
    a, _ = O.assign(X, C)
    idx = O.build(X, nlist, centroids=C, P=P, assignment=a)
    return X, Q, idx


def lib_index(X, idx, bq=4):
    from paper_2605_16007_amd import Index
    return Index.build(X, idx.nlist, bq=bq, centroids=idx.centroids, rotation=idx.P,
                       assignment=idx.assign.astype(np.int32))


def est_scale(rn2, vl, delta, squ, ip, pop, n_x, alpha, d):
    n_x = np.asarray(n_x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    inner = np.abs(vl) * np.abs(2 * pop - d) + delta * np.abs(2 * ip - squ)
    return rn2 + n_x * n_x + 2 * n_x * inner / (math.sqrt(d) * alpha)


def qu_boundary_eta(q, c, delta, d):
    """Bound (in y units) of the GPU's FP32 error on y = (r - v_l)/Delta."""
    if delta <= 0:
        return np.inf
    scale = float(np.linalg.norm(q)) + float(np.linalg.norm(c))
    return 8.0 * d * U32 * scale / delta + 1e-5


def set_diff_ok(gpu_ids, ref_ids, ref_val_of, boundary, tol_of):
    """Sets may differ only by elements whose reference value is within tol of
    the boundary value. Returns a list of violations."""
    g, r = set(int(x) for x in gpu_ids if x >= 0), set(int(x) for x in ref_ids if x >= 0)
    bad = []
    for x in g - r:
        if ref_val_of(x) > boundary + tol_of(x):
            bad.append(("extra", x, ref_val_of(x), boundary))
    for x in r - g:
        if ref_val_of(x) < boundary - tol_of(x):
            bad.append(("missing", x, ref_val_of(x), boundary))
    if len(g) != len(r):
        bad.append(("size", len(g), len(r)))
    return bad
