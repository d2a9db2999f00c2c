"""Pins of the CPU oracle against what the paper and mathematics fix.

Every oracle function is checked here against something other than itself:
hand-computed worked examples (tests/golden), pure-Python brute force on tiny
inputs, exact rational arithmetic, closed forms of the estimator, statistical
properties of the estimator over Haar-random rotations, and the reduction of
the whole search to exact kNN.
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle as O


# ---------------------------------------------------------------- fixtures

def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["worked_d4_identity.json", "worked_d4_hadamard.json"])
def test_worked_example(golden_dir, name):
    """Sec. 2.2.1-2.2.2 worked by hand (see the fixture's note)."""
    g = _load(golden_dir, name)
    D, bq = g["D"], g["bq"]
    P = np.array(g["P"], np.float64)
    c = np.array(g["c"], np.float32)[None, :]
    x = np.array(g["x"], np.float32)[None, :]
    q = np.array(g["q"], np.float32)
    codes, n_x, alpha = O.encode(x, c, np.array([0]), P)
    assert codes.tolist() == [g["code_bytes"]]
    assert n_x[0] == pytest.approx(g["n_x"], rel=1e-7)
    assert alpha[0] == pytest.approx(g["alpha"], rel=1e-7)
    r = O.rotate(q, P) - O.rotate(c[0], P)
    qu, vl, delta, squ = O.quantize(r, bq)
    assert qu.tolist() == g["qu"]
    assert vl == pytest.approx(g["v_l"], abs=1e-15)
    assert delta == pytest.approx(g["delta"], rel=1e-15)
    assert squ == g["sum_qu"]
    E, ip, pop = O.est_terms(codes, qu, vl, delta, D)
    assert ip.tolist() == [g["ip"]] and pop.tolist() == [g["pop"]]
    assert E[0] == pytest.approx(g["E"], rel=1e-14)
    assert float(r @ r) == pytest.approx(g["rnorm2"], rel=1e-15)
    est = O.estimate(float(r @ r), E, n_x, alpha, D)
    # factors are stored as FP32, so d_hat^2 carries their rounding
    assert est[0] == pytest.approx(g["d_hat2"], rel=1e-6)
    s = O.s_hat_unquantized(P, codes, (q - c[0]) / np.linalg.norm(q - c[0]), alpha, D)
    qn = float(np.linalg.norm(q.astype(np.float64) - c[0]))
    est_unq = qn ** 2 + float(n_x[0]) ** 2 - 2 * qn * float(n_x[0]) * s[0]
    assert est_unq == pytest.approx(g["d_hat2_unquantized"], rel=1e-6)
    assert float(np.sum((q.astype(np.float64) - x[0]) ** 2)) == g["d2_exact"]


# ---------------------------------------------------------------- IVF build

def test_assign_is_bruteforce_argmin_with_ties():
    """Sec. 2.1.2: each vector goes to its nearest centroid; ties -> lowest id."""
    rng = np.random.default_rng(1)
    X = rng.integers(-3, 4, size=(60, 3)).astype(np.float32)
    C = rng.integers(-3, 4, size=(9, 3)).astype(np.float32)
    C[5] = C[2]                          # an exact duplicate centroid: ties
    a, dmin = O.assign(X, C)
    for i in range(len(X)):
        best, bj = None, None
        for j in range(len(C)):
            d = sum((float(X[i, t]) - float(C[j, t])) ** 2 for t in range(3))
            if best is None or d < best:
                best, bj = d, j
        assert a[i] == bj and dmin[i] == best
    assert not np.any(a == 5)


def test_kmeanspp_picks_training_points_and_spreads():
    rng = np.random.default_rng(2)
    A = rng.normal(0, 1e-3, size=(20, 4))
    B = rng.normal(0, 1e-3, size=(20, 4)) + 1e6
    T = np.concatenate([A, B])
    for s in range(20):
        C = O.kmeanspp_init(T, 2, np.random.default_rng(s))
        for c in C:
            assert np.any(np.all(T == c, axis=1))
        # D^2 sampling must take the second centre from the far cluster
        assert (C[0, 0] > 1e5) != (C[1, 0] > 1e5)


def test_kmeans_objective_monotone_and_means():
    """Lloyd iterations never increase the objective; the result's centroids are
    the means of their assigned points (a fixed point)."""
    rng = np.random.default_rng(3)
    centres = rng.normal(0, 1, size=(8, 6))
    X = (centres[rng.integers(0, 8, 800)] + 0.3 * rng.normal(size=(800, 6))).astype(np.float32)
    trace = []
    C = O.kmeans(X, 8, np.random.default_rng(0), iters=50, restarts=2, trace=trace)
    for run in trace:
        assert all(b <= a * (1 + 1e-12) for a, b in zip(run, run[1:]))
    a, _ = O.assign(X, C)
    for j in range(8):
        m = a == j
        assert m.any()
        np.testing.assert_allclose(C[j], X[m].astype(np.float64).mean(axis=0), atol=1e-9)


def test_kmeans_recovers_separated_mixture():
    """Textbook special case: well-separated components are found exactly."""
    rng = np.random.default_rng(4)
    centres = np.eye(5) * 100.0
    lab = rng.integers(0, 5, 500)
    X = (centres[lab] + 0.01 * rng.normal(size=(500, 5))).astype(np.float32)
    C = O.kmeans(X, 5, np.random.default_rng(1), iters=25, restarts=3)
    d = O.sqdist(C, centres)
    assert np.all(np.min(d, axis=1) < 0.01)
    assert len(set(np.argmin(d, axis=1))) == 5


def test_kmeans_keeps_lowest_objective_restart():
    """With restarts, k-means keeps the run of lowest objective. Each restart
    draws only its own k-means++ seeding from the generator (the whole set is
    the training set here), so three restarts from one generator are the three
    single runs drawn from it in turn. Their objectives, computed here by brute
    force, differ, the best is not the last, and the result is the best run."""
    rng = np.random.default_rng(5)
    centres = rng.normal(0, 1, size=(12, 4)) * 3.0
    X = (centres[rng.integers(0, 12, 400)] + 0.8 * rng.normal(size=(400, 4))).astype(np.float32)

    def objective(C):
        return sum(min(sum((float(x[t]) - float(c[t])) ** 2 for t in range(4)) for c in C) for x in X)

    for seed in range(50):
        g = np.random.default_rng(seed)
        singles = [O.kmeans(X, 6, g, iters=3, restarts=1) for _ in range(3)]
        objs = [objective(C) for C in singles]
        best = int(np.argmin(objs))
        if best != 2 and len({round(o, 6) for o in objs}) == 3:
            break
    else:
        pytest.fail("no seed with distinct restart objectives and an earlier best")
    C = O.kmeans(X, 6, np.random.default_rng(seed), iters=3, restarts=3)
    np.testing.assert_array_equal(C, singles[best])
    assert objective(C) == min(objs)


def test_kmeans_seed_rows_subset():
    """With seed_rows the k-means++ centres come only from the evenly strided
    subset (row t * T // S, written out here with integer loops), and
    seed_rows >= T is the default procedure."""
    rng = np.random.default_rng(6)
    X = rng.normal(size=(300, 3)).astype(np.float32)
    T = X.astype(np.float64)
    S = 37
    sub = [T[(t * len(T)) // S] for t in range(S)]
    for seed in range(5):
        C = O.kmeanspp_init(np.array(sub), 5, np.random.default_rng(seed))
        for c in C:
            assert any(np.array_equal(c, r) for r in sub)
        a = O.kmeans(X, 5, np.random.default_rng(seed), iters=0, restarts=1, seed_rows=S)
        np.testing.assert_array_equal(a, C)  # zero Lloyd steps: the seeds themselves
    a = O.kmeans(X, 5, np.random.default_rng(9), iters=4, restarts=2, seed_rows=10_000)
    b = O.kmeans(X, 5, np.random.default_rng(9), iters=4, restarts=2)
    np.testing.assert_array_equal(a, b)


def test_kmeans_random_init_rows():
    """init="random": the starting centroids are distinct training rows (zero
    Lloyd steps return them), and Lloyd steps from them never raise the
    objective."""
    rng = np.random.default_rng(8)
    X = rng.integers(0, 50, size=(200, 2)).astype(np.float32)
    C = O.kmeans(X, 7, np.random.default_rng(1), iters=0, restarts=1, init="random")
    rows = {tuple(r) for r in X.astype(np.float64).tolist()}
    assert len({tuple(c) for c in C.tolist()}) == 7
    assert all(tuple(c) in rows for c in C.tolist())
    trace = []
    O.kmeans(X, 7, np.random.default_rng(1), iters=20, restarts=2, init="random", trace=trace)
    for run in trace:
        assert all(b <= a * (1 + 1e-12) for a, b in zip(run, run[1:]))


def test_kmeans_empty_cluster_reseed():
    """An empty cluster is moved onto the point farthest from its centroid."""
    T = np.array([[0.0], [1.0], [10.0]])
    C0 = np.array([[0.5], [100.0]])
    a, dmin = O.assign(T, C0)
    assert (a == 1).sum() == 0
    C1 = O.lloyd_update(T, a, C0, dmin)
    assert C1[1, 0] == 10.0
    assert C1[0, 0] == pytest.approx(11.0 / 3.0)


@pytest.mark.parametrize("d", [8, 16, 96, 128])
def test_rotation_is_orthogonal(d):
    """Sec. 2.2.1: P is orthogonal, so it preserves norms (used in Sec. 3.2.2)."""
    P = O.random_orthogonal(d, np.random.default_rng(d))
    assert np.max(np.abs(P.T @ P - np.eye(d))) <= 1e-12
    P32 = P.astype(np.float32).astype(np.float64)
    assert np.max(np.abs(P32.T @ P32 - np.eye(d))) <= 1e-6
    q = np.random.default_rng(5).normal(size=(50, d))
    nq = np.linalg.norm(q, axis=1)
    assert np.all(np.abs(np.linalg.norm(O.rotate(q, P32), axis=1) - nq) <= 1e-6 * nq)


def test_rotation_is_haar():
    """Haar-random columns are uniform on the sphere: E[P_ij^2] = 1/D, and the
    determinant takes both signs."""
    d = 8
    sq, dets = [], []
    for s in range(800):
        P = O.random_orthogonal(d, np.random.default_rng(1000 + s))
        sq.append(P[0, 0] ** 2)
        dets.append(np.sign(np.linalg.det(P)))
    m = np.mean(sq)
    se = np.std(sq) / math.sqrt(len(sq))
    assert abs(m - 1.0 / d) < 4 * se
    assert 0.4 < np.mean(np.array(dets) > 0) < 0.6


# ---------------------------------------------------------------- encoding

def test_pack_bits_lsb_first():
    bits = np.zeros((1, 12), np.uint8)
    bits[0, [0, 3, 8, 11]] = 1
    assert O.pack_bits(bits).tolist() == [[0b00001001, 0b00001001]]
    np.testing.assert_array_equal(O.unpack_bits(O.pack_bits(bits), 12), bits)


@pytest.mark.parametrize("d", [16, 96, 128, 960])
def test_alpha_identity_and_range(d):
    """Eq. rabitq-alpha: <P b / sqrt(D), u_x> equals ||P^T u_x||_1 / sqrt(D),
    and alpha lies in [1/sqrt(D), 1]; for Gaussian residuals its mean is near
    sqrt(2/pi)."""
    rng = np.random.default_rng(d)
    P = O.random_orthogonal(d, rng) if d <= 128 else np.linalg.qr(rng.normal(size=(d, d)))[0]
    X = rng.normal(size=(400, d)).astype(np.float32)
    C = np.zeros((1, d), np.float32)
    codes, n_x, alpha = O.encode(X, C, np.zeros(400, np.int64), P)
    b = 2.0 * O.unpack_bits(codes, d).astype(np.float64) - 1.0
    u = X.astype(np.float64) / np.linalg.norm(X.astype(np.float64), axis=1, keepdims=True)
    lhs = np.einsum("ij,ij->i", (P @ b.T).T / math.sqrt(d), u)
    np.testing.assert_allclose(lhs, alpha.astype(np.float64), rtol=1e-6)
    assert np.all(alpha >= 1 / math.sqrt(d) - 1e-7) and np.all(alpha <= 1 + 1e-7)
    assert abs(alpha.mean() - math.sqrt(2 / math.pi)) < 0.03
    np.testing.assert_allclose(n_x, np.linalg.norm(X.astype(np.float64), axis=1), rtol=1e-7)


def test_encode_degenerate_zero_residual():
    """n_x = 0 (a vector equal to its centroid): alpha = 1, all-ones code."""
    d = 16
    P = O.random_orthogonal(d, np.random.default_rng(0))
    X = np.ones((2, d), np.float32)
    X[1, 0] = 2.0
    codes, n_x, alpha = O.encode(X, np.ones((1, d), np.float32), np.zeros(2, np.int64), P)
    assert n_x[0] == 0.0 and alpha[0] == 1.0
    assert codes[0].tolist() == [255, 255]
    assert n_x[1] == 1.0


def test_encode_sign_matches_rotation_bruteforce():
    """Codes are the signs of P^T (x - c), written out as plain loops."""
    d = 12
    rng = np.random.default_rng(7)
    P = O.random_orthogonal(d, rng)
    X = rng.normal(size=(5, d)).astype(np.float32)
    C = rng.normal(size=(2, d)).astype(np.float32)
    a = np.array([0, 1, 1, 0, 1])
    codes, _, _ = O.encode(X, C, a, P)
    for i in range(5):
        z = [sum(P[t, j] * (float(X[i, t]) - float(C[a[i], t])) for t in range(d)) for j in range(d)]
        byte = [0] * 2
        for j in range(d):
            if z[j] >= 0:
                byte[j >> 3] |= 1 << (j & 7)
        assert codes[i].tolist() == byte


# ---------------------------------------------------------------- query side

def test_quantize_bounds_and_degenerate():
    rng = np.random.default_rng(8)
    for bq in (1, 2, 4, 8):
        top = (1 << bq) - 1
        r = rng.normal(size=128)
        qu, vl, delta, squ = O.quantize(r, bq)
        assert qu.min() == 0 and qu.max() == top
        assert vl == r.min() and delta == pytest.approx((r.max() - r.min()) / top)
        assert np.all(np.abs(r - (vl + delta * qu)) <= delta / 2 * (1 + 1e-12))
        assert squ == qu.sum()
    qu, vl, delta, squ = O.quantize(np.full(16, 3.5), 4)
    assert delta == 0.0 and vl == 3.5 and squ == 0 and not qu.any()


def test_quantize_round_half_up_bruteforce():
    """Rounding is floor(y + 1/2), checked against exact rationals."""
    r = np.array([0.0, 1.0, 2.0, 3.0, 0.5, 1.5, 2.5, 0.25], np.float64)
    qu, vl, delta, _ = O.quantize(r, 2)          # Delta = 1
    exp = [math.floor(Fraction(v) + Fraction(1, 2)) for v in r]
    assert qu.tolist() == exp


def test_integer_ip_two_routes_and_bruteforce():
    """Sec. 2.2.2: the bitwise (bit-plane popcount) route and a dense product of
    small integers give the same integer inner products, equal to a pure-Python
    double loop."""
    rng = np.random.default_rng(9)
    for d in (8, 13, 96, 128, 960):
        bits = rng.integers(0, 2, size=(40, d)).astype(np.uint8)
        codes = O.pack_bits(bits)
        for bq in (1, 4, 8):
            qu = rng.integers(0, 1 << bq, size=d)
            a = O.ip_dense(codes, qu, d)
            b = O.ip_bitplanes(codes, qu, d, bq)
            np.testing.assert_array_equal(a, b)
            if d <= 13:
                for i in range(40):
                    assert a[i] == sum(int(bits[i, t]) * int(qu[t]) for t in range(d))


def test_E_identity_exact_rationals():
    """E = sum_d b_d (v_l + Delta qu_d) = 2 Delta ip + 2 v_l pop - Delta sum(qu) - D v_l,
    in exact rational arithmetic; the oracle's FP64 E agrees to rounding."""
    rng = np.random.default_rng(10)
    d, bq = 24, 4
    for _ in range(20):
        bits = rng.integers(0, 2, size=(1, d)).astype(np.uint8)
        codes = O.pack_bits(bits)
        r = rng.normal(size=d)
        qu, vl, delta, squ = O.quantize(r, bq)
        Fv, Fd = Fraction(vl), Fraction(delta)
        lhs = sum((2 * int(bits[0, t]) - 1) * (Fv + Fd * int(qu[t])) for t in range(d))
        ip = sum(int(bits[0, t]) * int(qu[t]) for t in range(d))
        pop = int(bits.sum())
        rhs = 2 * Fd * ip + 2 * Fv * pop - Fd * squ - d * Fv
        assert lhs == rhs
        E, ip_o, pop_o = O.est_terms(codes, qu, vl, delta, d)
        assert ip_o[0] == ip and pop_o[0] == pop
        assert abs(E[0] - float(lhs)) <= 1e-12 * (abs(vl) * d + delta * 15 * d)


def test_quantisation_error_bound():
    """|E - sum_d b_d r_d| <= D Delta / 2 (each dimension is off by <= Delta/2)."""
    rng = np.random.default_rng(11)
    d = 128
    bits = rng.integers(0, 2, size=(200, d)).astype(np.uint8)
    codes = O.pack_bits(bits)
    b = 2.0 * bits - 1.0
    for _ in range(10):
        r = rng.normal(size=d) * rng.uniform(0.1, 10)
        qu, vl, delta, _ = O.quantize(r, 4)
        E, _, _ = O.est_terms(codes, qu, vl, delta, d)
        assert np.all(np.abs(E - b @ r) <= d * delta / 2 * (1 + 1e-12))


def test_estimator_exact_on_ray():
    """Closed form of Eqs. rabitq-ip-estimator / approx-dist: if q lies on the
    ray c + t (x - c), then P^T u_q = sign(t) P^T u_x, so <b, z_q> =
    sign(t) ||z_x||_1 and s_hat = sign(t) exactly: d_hat^2 equals the exact
    d^2 = (||q-c|| - sign(t) ||x-c||)^2. With q = x, d_hat^2 = 0."""
    d = 64
    rng = np.random.default_rng(12)
    P = O.random_orthogonal(d, rng)
    c = rng.normal(size=(1, d)).astype(np.float32)
    x = rng.normal(size=(1, d)).astype(np.float32)
    codes, n_x, alpha = O.encode(x, c, np.array([0]), P)
    for t in (-2.0, -0.5, 0.3, 1.0, 3.0):
        q = c[0].astype(np.float64) + t * (x[0].astype(np.float64) - c[0])
        qn = np.linalg.norm(q - c[0])
        s = O.s_hat_unquantized(P, codes, (q - c[0]) / qn, alpha.astype(np.float64), d)
        # alpha is stored in FP32, so s_hat is sign(t) to FP32 precision
        assert s[0] == pytest.approx(math.copysign(1.0, t), rel=1e-6)
        exact = float(np.sum((q - x[0].astype(np.float64)) ** 2))
        est = qn ** 2 + float(n_x[0]) ** 2 - 2 * qn * float(n_x[0]) * s[0]
        assert est == pytest.approx(exact, rel=1e-5, abs=1e-5 * (qn ** 2 + float(n_x[0]) ** 2))
        # and through the quantised pipeline with many bits the error is tiny
        r = O.rotate(q, P) - O.rotate(c[0].astype(np.float64), P)
        qu, vl, delta, _ = O.quantize(r, 20)
        E, _, _ = O.est_terms(codes, qu, vl, delta, d)
        est_q = O.estimate(float(r @ r), E, n_x, alpha, d)[0]
        assert est_q == pytest.approx(exact, abs=1e-4 * (qn ** 2 + float(n_x[0]) ** 2))


def _haar_two_frame_P(u1, u2, rng):
    """A full orthogonal P whose action on span(u1, u2) has the Haar law.

    For Haar-random P, (P^T u1, P^T u2) of an orthonormal pair is a uniformly
    random orthonormal 2-frame (f1, f2); QR of a D x 2 Gaussian matrix with the
    signs of R's diagonal folded in draws exactly such a frame. P^T = H2 H1 with
    two Householder reflections: H1 takes u1 to f1, H2 takes H1 u2 to f2 and
    fixes f1 (both are orthogonal to f1). The estimator sees P only through
    P^T x and P^T q for x, q in span(u1, u2), so its law under this P equals its
    law under a Haar P, at O(D^2) cost per draw instead of a D x D QR.
    P = H1 H2 = I + U V^T, a rank-two update."""
    d = len(u1)
    F, R = np.linalg.qr(rng.standard_normal((d, 2)))
    F = F * np.sign(np.diag(R))[None, :]
    w1 = u1 - F[:, 0]
    w1 /= np.linalg.norm(w1)
    y = u2 - 2.0 * (w1 @ u2) * w1
    w2 = y - F[:, 1]
    w2 /= np.linalg.norm(w2)
    U = np.stack([w1, w2], 1)
    V = np.stack([-2.0 * w1 + 4.0 * (w1 @ w2) * w2, -2.0 * w2], 1)
    P = U @ V.T
    P[np.diag_indices(d)] += 1.0
    np.testing.assert_allclose(u1 @ P, F[:, 0], atol=1e-12)
    np.testing.assert_allclose(u2 @ P, F[:, 1], atol=1e-12)
    return P


def _shat_errors(d, trials, rng, draw_P):
    """s_hat - <u_x, u_q> over `trials` draws of P, for a fixed pair at cos 0.6."""
    ux, w, uq = _pair_with_cos_basis(d, 0.6, rng)
    errs = np.empty(trials)
    for t in range(trials):
        P = draw_P(ux, w, rng)
        codes, _, _ = O.encode(ux[None, :].astype(np.float32), np.zeros((1, d), np.float32),
                               np.array([0]), P)
        z = ux @ P
        alpha64 = np.sum(np.abs(z)) / (math.sqrt(d) * np.linalg.norm(z))
        errs[t] = O.s_hat_unquantized(P, codes, uq, np.array([alpha64]), d)[0] - float(ux @ uq)
    return errs


def _pair_with_cos_basis(d, cos, rng):
    u = rng.normal(size=d)
    u /= np.linalg.norm(u)
    w = rng.normal(size=d)
    w -= (w @ u) * u
    w /= np.linalg.norm(w)
    return u, w, cos * u + math.sqrt(1 - cos * cos) * w


def test_estimator_unbiased_with_oracle_rotation():
    """RaBitQ's unbiasedness (cited in Sec. 2.2) through the oracle's own Haar
    generator: over 2000 draws of P the mean error of s_hat is within 3
    standard errors of zero."""
    rng = np.random.default_rng(13)
    for d in (32, 64):
        errs = _shat_errors(d, 2000, rng, lambda u1, u2, g: O.random_orthogonal(len(u1), g))
        se = errs.std() / math.sqrt(len(errs))
        assert abs(errs.mean()) <= 3.0 * se, (d, errs.mean(), se)


def test_estimator_unbiased_and_sqrt_d_error():
    """RaBitQ's guarantees (cited in Sec. 2.2): over Haar-random P the
    estimator s_hat of <u_x, u_q> is unbiased (|mean error| <= 3 standard
    errors over 2000 draws), and its error shrinks as O(1/sqrt(D)):
    std(s_hat - s) sqrt(D) is flat within +-15% from D = 32 to D = 960."""
    rng = np.random.default_rng(17)
    scaled = []
    for d in (32, 64, 128, 256, 960):
        errs = _shat_errors(d, 2000, rng, _haar_two_frame_P)
        se = errs.std() / math.sqrt(len(errs))
        assert abs(errs.mean()) <= 3.0 * se, (d, errs.mean(), se)
        scaled.append(errs.std() * math.sqrt(d))
    mid = math.sqrt(max(scaled) * min(scaled))
    assert all(abs(v / mid - 1.0) <= 0.15 for v in scaled), scaled


def test_two_frame_rotation_matches_haar_law():
    """The two-frame P above has the law of a Haar P on the pair's plane: the
    first two moments of (P^T u1)_0 and of <P^T u1, e_0><P^T u2, e_0> agree
    with those under the oracle's Haar generator (E = 0, E[z^2] = 1/D)."""
    d, trials = 16, 4000
    rng = np.random.default_rng(21)
    u1, u2, _ = _pair_with_cos_basis(d, 0.0, rng)
    for draw in (_haar_two_frame_P, lambda a, b, g: O.random_orthogonal(d, g)):
        z1 = np.empty(trials)
        z12 = np.empty(trials)
        for t in range(trials):
            P = draw(u1, u2, rng)
            np.testing.assert_allclose(P.T @ P, np.eye(d), atol=1e-12)
            a, b = u1 @ P, u2 @ P
            z1[t], z12[t] = a[0], a[0] * b[0]
        assert abs(z1.mean()) <= 4.0 * z1.std() / math.sqrt(trials)
        assert abs(np.mean(z1 ** 2) * d - 1.0) <= 0.06
        # E[z1 z2] = 0 for orthogonal u1, u2 and E[(z1 z2)^2] = 1 / (D (D + 2))
        assert abs(z12.mean()) <= 4.0 * z12.std() / math.sqrt(trials)
        assert abs(np.mean(z12 ** 2) * d * (d + 2) - 1.0) <= 0.1


# ---------------------------------------------------------------- selection

def test_probe_bruteforce_with_ties():
    rng = np.random.default_rng(14)
    C = rng.integers(-2, 3, size=(30, 3)).astype(np.float32)
    for _ in range(10):
        q = rng.integers(-2, 3, size=3).astype(np.float32)
        ids, dist = O.probe(q, C, 7)
        full = sorted(((sum((float(q[t]) - float(C[j, t])) ** 2 for t in range(3)), j)
                       for j in range(30)))
        assert ids.tolist() == [j for _, j in full[:7]]
        assert dist.tolist() == [v for v, _ in full[:7]]


def test_topk_lex_and_padding():
    rng = np.random.default_rng(15)
    v = rng.integers(0, 5, size=50).astype(np.float64)
    ids = rng.permutation(50)
    tv, ti = O.topk_lex(v, ids, 12)
    ref = sorted(zip(v.tolist(), ids.tolist()))[:12]
    assert list(zip(tv.tolist(), ti.tolist())) == ref
    tv, ti = O.topk_lex(v[:3], ids[:3], 5)
    assert ti[3:].tolist() == [-1, -1] and np.all(np.isinf(tv[3:]))


def test_bruteforce_knn_loops():
    rng = np.random.default_rng(16)
    X = rng.integers(0, 4, size=(40, 3)).astype(np.float32)
    Q = rng.integers(0, 4, size=(5, 3)).astype(np.float32)
    ids, d = O.brute_force_knn(X, Q, 6, chunk=7)
    for qi in range(5):
        full = sorted((sum((float(Q[qi, t]) - float(X[i, t])) ** 2 for t in range(3)), i)
                      for i in range(40))[:6]
        assert ids[qi].tolist() == [i for _, i in full]
        assert d[qi].tolist() == [v for v, _ in full]


def test_rerank_bruteforce():
    rng = np.random.default_rng(17)
    X = rng.normal(size=(30, 5)).astype(np.float32)
    q = rng.normal(size=5).astype(np.float32)
    cand = np.array([3, 7, 1, 29, 11, -1, -1])
    d, i = O.rerank(q, X, cand, 3)
    full = sorted((float(np.sum((X[j].astype(np.float64) - q) ** 2)), j) for j in [3, 7, 1, 29, 11])
    assert i.tolist() == [j for _, j in full[:3]]
    d, i = O.rerank(q, X, cand, 8)
    assert i[5:].tolist() == [-1, -1, -1]


# ---------------------------------------------------------------- whole search

def test_search_reduces_to_exact_knn():
    """With every list probed and every candidate re-ranked, IVF-RaBitQ search
    is exact kNN (Sec. 2.1.1 problem definition)."""
    rng = np.random.default_rng(18)
    X = rng.normal(size=(600, 16)).astype(np.float32)
    Q = rng.normal(size=(8, 16)).astype(np.float32)
    idx = O.build(X, 8, rng=np.random.default_rng(0), kmeans_iters=5, kmeans_restarts=1)
    ids, d = O.search(idx, X, Q, nprobe=8, k=10, rerank_n=600)
    ids_bf, d_bf = O.brute_force_knn(X, Q, 10)
    np.testing.assert_array_equal(ids, ids_bf)
    np.testing.assert_allclose(d, d_bf, rtol=1e-12)


def test_search_stages_consistent():
    """Stage outputs agree with the stand-alone definitions: probes are the
    nprobe nearest lists; every candidate set is the lexicographic top-R of all
    estimated distances of the probed lists."""
    rng = np.random.default_rng(19)
    X = rng.normal(size=(900, 32)).astype(np.float32)
    Q = rng.normal(size=(4, 32)).astype(np.float32)
    idx = O.build(X, 12, rng=np.random.default_rng(1), kmeans_iters=5, kmeans_restarts=1)
    ids, d, st = O.search(idx, X, Q, nprobe=4, k=5, rerank_n=40, stages=True)
    for qi in range(4):
        full = sorted((float(np.sum((idx.centroids[j].astype(np.float64) - Q[qi]) ** 2)), j)
                      for j in range(12))
        assert st["probes"][qi].tolist() == [j for _, j in full[:4]]
        allv = np.concatenate([pl["est"] for pl in st["per_list"][qi]])
        alli = np.concatenate([pl["ids"] for pl in st["per_list"][qi]])
        ref = sorted(zip(allv.tolist(), alli.tolist()))[:40]
        assert st["cand_ids"][qi].tolist() == [i for _, i in ref]
        # every probed list's members are assigned to it
        for j, pl in zip(st["probes"][qi], st["per_list"][qi]):
            assert np.all(idx.assign[pl["ids"]] == j)
    assert np.all(np.diff(d, axis=1) >= 0)


def test_recall_small_mixture():
    """A quality check on a small Gaussian mixture: recall@10 is high once
    enough candidates are re-ranked."""
    from synth import get, database, queries
    w = get("mixture128", n=20_000, nq=20, nlist=64)
    X = database(w)
    Q = queries(w)
    idx = O.build(X, 64, rng=np.random.default_rng(0), kmeans_iters=10, kmeans_restarts=1)
    ids, _ = O.search(idx, X, Q, nprobe=8, k=10, rerank_n=200)
    gt, _ = O.brute_force_knn(X, Q, 10)
    rec = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(ids.tolist(), gt.tolist())])
    assert rec >= 0.9, rec


# ------------------------------------------- unquantised-query estimator

def test_unquantized_E_exact_rationals():
    """E = sum_d b_d r_d and ip = sum_d b01_d r_d for an unquantised residual
    (Eq. rabitq-ip-estimator without query SQ), against exact rational sums on
    a tiny input whose values are exact binary fractions."""
    rng = np.random.default_rng(31)
    d = 13
    for _ in range(20):
        bits = rng.integers(0, 2, size=(3, d)).astype(np.uint8)
        r = rng.integers(-64, 65, size=d) / 8.0
        E, ip, pop = O.est_terms_unquantized(O.pack_bits(bits), r, d)
        for v in range(3):
            e = sum(Fraction(r[t]) * (1 if bits[v, t] else -1) for t in range(d))
            i = sum(Fraction(r[t]) for t in range(d) if bits[v, t])
            assert Fraction(E[v]) == e and Fraction(ip[v]) == i
            assert pop[v] == int(bits[v].sum())


def test_unquantized_E_is_scaled_shat():
    """E / (sqrt(D) alpha ||q - c||) is the estimator s_hat of Eq.
    rabitq-ip-estimator: the residual route (P^T q - P^T c) and the unit-vector
    route (P^T u_q) agree."""
    rng = np.random.default_rng(32)
    d = 40
    P = O.random_orthogonal(d, rng)
    c = rng.normal(size=(1, d)).astype(np.float32)
    X = rng.normal(size=(30, d)).astype(np.float32)
    codes, n_x, alpha = O.encode(X, c, np.zeros(30, np.int64), P)
    q = rng.normal(size=d).astype(np.float32)
    r = O.rotate(q, P) - O.rotate(c[0], P)
    E, _, _ = O.est_terms_unquantized(codes, r, d)
    qc = q.astype(np.float64) - c[0]
    s = O.s_hat_unquantized(P, codes, qc / np.linalg.norm(qc), alpha.astype(np.float64), d)
    np.testing.assert_allclose(E / (math.sqrt(d) * alpha.astype(np.float64) * np.linalg.norm(qc)), s,
                               rtol=1e-12, atol=1e-12)


def test_unquantized_search_exact_on_ray():
    """Closed form: for q on the ray c + t (x - c) the unquantised estimate is
    the exact distance (s_hat = sign(t)); checked through the search's own
    stage outputs."""
    rng = np.random.default_rng(33)
    d = 24
    X = rng.normal(size=(50, d)).astype(np.float32)
    idx = O.build(X, 1, centroids=np.zeros((1, d), np.float32), P=O.random_orthogonal(d, rng))
    for t in (-1.5, 0.4, 2.0):
        q = (t * X[7].astype(np.float64)).astype(np.float32)
        _, _, st = O.search(idx, X, q[None, :], 1, 1, 50, stages=True, unquantized=True)
        pl = st["per_list"][0][0]
        pos = int(np.flatnonzero(pl["ids"] == 7)[0])
        exact = float(np.sum((q.astype(np.float64) - X[7]) ** 2))
        scale = float(np.sum(q.astype(np.float64) ** 2) + np.sum(X[7].astype(np.float64) ** 2))
        assert abs(pl["est"][pos] - exact) <= 1e-5 * scale


def test_quantized_estimate_tends_to_unquantized():
    """|E_q - E| <= D Delta / 2 for the B_q-bit query against the unquantised
    one, and the difference vanishes as B_q grows."""
    rng = np.random.default_rng(34)
    d = 96
    codes = O.pack_bits(rng.integers(0, 2, size=(100, d)).astype(np.uint8))
    r = rng.normal(size=d)
    E, _, _ = O.est_terms_unquantized(codes, r, d)
    prev = None
    for bq in (2, 4, 8, 16, 24):
        qu, vl, delta, _ = O.quantize(r, bq)
        Eq, _, _ = O.est_terms(codes, qu, vl, delta, d)
        err = np.max(np.abs(Eq - E))
        assert err <= d * delta / 2 * (1 + 1e-9)
        if prev is not None:
            assert err < prev
        prev = err
    assert prev < 1e-5


def test_unquantized_search_reduces_to_exact_knn():
    """Every list probed and every candidate re-ranked: exact kNN."""
    rng = np.random.default_rng(35)
    X = rng.normal(size=(500, 12)).astype(np.float32)
    Q = rng.normal(size=(6, 12)).astype(np.float32)
    idx = O.build(X, 6, rng=np.random.default_rng(0), kmeans_iters=5, kmeans_restarts=1)
    ids, d = O.search(idx, X, Q, nprobe=6, k=8, rerank_n=500, unquantized=True)
    ids_bf, d_bf = O.brute_force_knn(X, Q, 8)
    np.testing.assert_array_equal(ids, ids_bf)
    np.testing.assert_allclose(d, d_bf, rtol=1e-12)


# ------------------------------------------------------------ IVF-Flat

def test_ivf_flat_bruteforce_loops():
    """IVF-Flat (Sec. 2.1.2 query processing over full-precision vectors):
    pure-Python loops over the probed lists, distances as exact sums of
    squares of small integers, ties by id, padding when the lists hold fewer
    than k vectors."""
    rng = np.random.default_rng(36)
    X = rng.integers(-3, 4, size=(40, 3)).astype(np.float32)
    C = rng.integers(-3, 4, size=(5, 3)).astype(np.float32)
    a, _ = O.assign(X, C)
    idx = O.build(X, 5, centroids=C, P=np.eye(3), assignment=a)
    Q = rng.integers(-3, 4, size=(6, 3)).astype(np.float32)
    for nprobe, k in ((1, 4), (2, 7), (5, 40), (1, 50)):
        ids, dd = O.ivf_flat_search(idx, X, Q, nprobe, k)
        for qi in range(len(Q)):
            cd = sorted((sum((float(Q[qi, t]) - float(C[j, t])) ** 2 for t in range(3)), j) for j in range(5))
            probed = {j for _, j in cd[:nprobe]}
            cand = sorted((sum((float(X[i, t]) - float(Q[qi, t])) ** 2 for t in range(3)), i)
                          for i in range(len(X)) if int(a[i]) in probed)[:k]
            want_i = [i for _, i in cand] + [-1] * (k - len(cand))
            want_d = [v for v, _ in cand] + [math.inf] * (k - len(cand))
            assert ids[qi].tolist() == want_i
            assert dd[qi].tolist() == want_d


def test_ivf_flat_all_lists_is_exact_knn():
    rng = np.random.default_rng(37)
    X = rng.normal(size=(700, 10)).astype(np.float32)
    Q = rng.normal(size=(5, 10)).astype(np.float32)
    idx = O.build(X, 9, rng=np.random.default_rng(0), kmeans_iters=4, kmeans_restarts=1)
    ids, d = O.ivf_flat_search(idx, X, Q, 9, 12)
    ids_bf, d_bf = O.brute_force_knn(X, Q, 12)
    np.testing.assert_array_equal(ids, ids_bf)
    np.testing.assert_allclose(d, d_bf, rtol=1e-12)
